// hop.hip -- the stencil kernels of the Schur complement D_S = A_ee - H_eo A_oo^-1 H_oe
// (eq. 3 with D_eo = -H_eo, D_oe = -H_oe, D_ee = A_ee, D_oo = A_oo).
//
// One thread per output site.  All fields are structure-of-arrays per parity
// (row stride V/2), so every load of a neighbour row, a link entry or a clover
// slot is one coalesced 8- or 16-byte access per lane.  Each site carries its
// eight incident links (forward U_mu(x) and pre-daggered backward U_mu(x-mu)^H),
// so link reads never gather.  Kernel A (odd output) and kernel B (even output)
// are one template with different epilogues (HopMode).
#include "ddq_internal.h"

namespace ddq {

template <int MU, typename R>
__device__ __forceinline__ void neighbours(const Geo& g, const Site& s, int& jf, int& jb, R& bf, R& bb) {
  bf = R(1);
  bb = R(1);
  if (MU == 0) {
    int base = s.i - (s.x >> 1);
    int xf = (s.x + 1 == g.L[0]) ? 0 : s.x + 1;
    int xb = (s.x == 0) ? g.L[0] - 1 : s.x - 1;
    jf = base + (xf >> 1);
    jb = base + (xb >> 1);
  } else if (MU == 1) {
    jf = (s.y + 1 == g.L[1]) ? s.i - (g.L[1] - 1) * g.sY : s.i + g.sY;
    jb = (s.y == 0) ? s.i + (g.L[1] - 1) * g.sY : s.i - g.sY;
  } else if (MU == 2) {
    jf = (s.z + 1 == g.L[2]) ? s.i - (g.L[2] - 1) * g.sZ : s.i + g.sZ;
    jb = (s.z == 0) ? s.i + (g.L[2] - 1) * g.sZ : s.i - g.sZ;
  } else {
    bool wf = (s.t + 1 == g.L[3]);
    bool wb = (s.t == 0);
    jf = wf ? s.i - (g.L[3] - 1) * g.sT : s.i + g.sT;
    jb = wb ? s.i + (g.L[3] - 1) * g.sT : s.i - g.sT;
    if (g.antiperiodic) {
      bf = wf ? R(-1) : R(1);
      bb = wb ? R(-1) : R(1);
    }
  }
}

// Orders one hop before the next: the accumulator is routed through an empty
// volatile asm, so the hop's arithmetic has to finish here, and the memory
// clobber keeps the next hop's loads below.  Without it the instruction
// selector lifts all 96 neighbour loads to the top and spills them.
template <typename R>
__device__ __forceinline__ void hop_fence(Spinor<R>& acc) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc.c[sp][c].r), "+v"(acc.c[sp][c].i)::"memory");
  __builtin_amdgcn_sched_barrier(0);
}

template <typename R>
__device__ __forceinline__ void scale_half(Half<R>& h, R f) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) h.c[s][c] = f * h.c[s][c];
}

// acc += (1 + sf g_mu) U_mu(x) in(x+mu) + (1 + sb g_mu) U_mu(x-mu)^H in(x-mu)
template <int MU, typename R>
__device__ __forceinline__ void hop_dir(Spinor<R>& acc, const HopArgs<R>& a, const Rows<R>& in,
                                        const Site& s, R sf, R sb) {
  const int vh = a.g.Vh;
  int jf, jb;
  R bf, bb;
  neighbours<MU, R>(a.g, s, jf, jb, bf, bb);
  {
    Spinor<R> p = load_spinor<R>(in, jf);
    Half<R> h = project<MU, R>(p, sf);
    Half<R> uh = link_mul<R>(rows<R>(a.links + (size_t)MU * 9 * vh, 9, vh), s.i, h);
    if (MU == 3) scale_half(uh, bf);
    accumulate<MU, R>(acc, uh, sf);
  }
  hop_fence<R>(acc);
  {
    Spinor<R> p = load_spinor<R>(in, jb);
    Half<R> h = project<MU, R>(p, sb);
    Half<R> uh = link_mul<R>(rows<R>(a.links + (size_t)(4 + MU) * 9 * vh, 9, vh), s.i, h);
    if (MU == 3) scale_half(uh, bb);
    accumulate<MU, R>(acc, uh, sb);
  }
  hop_fence<R>(acc);
}

// register budget: waves per SIMD the scheduler must keep resident
#ifndef DDQ_WAVES_F64
#define DDQ_WAVES_F64 2
#endif
#ifndef DDQ_WAVES_F32
#define DDQ_WAVES_F32 4
#endif
template <typename R> struct HOP_WAVES { static constexpr int value = DDQ_WAVES_F32; };
template <> struct HOP_WAVES<double> { static constexpr int value = DDQ_WAVES_F64; };

template <typename R, int MODE, bool DAG>
__global__ void __launch_bounds__(HOP_BLOCK) __attribute__((amdgpu_waves_per_eu(HOP_WAVES<R>::value)))
hop_kernel(HopArgs<R> a) {
  const int vh = a.g.Vh;
  const int i = xcd_block(a.nblk) * HOP_BLOCK + (int)threadIdx.x;
  if (i >= vh) return;
  const size_t roff = (size_t)blockIdx.y * (size_t)a.rhs_stride;
  const Rows<R> in = rows<R>(a.in + roff, 12, vh);
  const Rows<R> cl = rows<R>(a.clov, 36, vh);
  const Site s = decode(a.g, i, a.p_out);
  // D: forward (1 - g), backward (1 + g).  D^H = g5 D g5 flips both projectors.
  const R sf = DAG ? R(1) : R(-1);
  const R sb = -sf;

  Spinor<R> acc;
  zero(acc);
  hop_dir<0, R>(acc, a, in, s, sf, sb);
  hop_dir<1, R>(acc, a, in, s, sf, sb);
  hop_dir<2, R>(acc, a, in, s, sf, sb);
  hop_dir<3, R>(acc, a, in, s, sf, sb);
  // h = 1/2 acc
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.c[sp][c] = R(0.5) * acc.c[sp][c];

  const Rows<R> out = rows<R>(a.out + roff, 12, vh);  // may alias a.x (in-place Richardson)
  if constexpr (MODE == M_HOP_CLINV) {
    store_spinor<R>(out, i, clover_mul<R>(cl, i, acc));
  } else if constexpr (MODE == M_RECON) {
    Spinor<R> bb = load_spinor<R>(rows<R>(a.b + roff, 12, vh), i);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) bb.c[sp][c] = bb.c[sp][c] + acc.c[sp][c];
    store_spinor<R>(out, i, clover_mul<R>(cl, i, bb));
  } else if constexpr (MODE == M_APPLY) {
    Spinor<R> cx = clover_mul<R>(cl, i, load_spinor<R>(rows<R>(a.x + roff, 12, vh), i));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) cx.c[sp][c] = cx.c[sp][c] - acc.c[sp][c];
    store_spinor<R>(out, i, cx);
  } else if constexpr (MODE == M_RICH) {
    Spinor<R> xx = load_spinor<R>(rows<R>(a.x + roff, 12, vh), i);
    Spinor<R> bb = load_spinor<R>(rows<R>(a.b + roff, 12, vh), i);
    Spinor<R> cx = clover_mul<R>(cl, i, xx);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        cpx<R> r = bb.c[sp][c] - cx.c[sp][c] + acc.c[sp][c];
        xx.c[sp][c] = xx.c[sp][c] + a.omega * r;
      }
    store_spinor<R>(out, i, xx);
  } else if constexpr (MODE == M_RESID) {
    Spinor<R> bb = load_spinor<R>(rows<R>(a.b + roff, 12, vh), i);
    Spinor<R> cx = clover_mul<R>(cl, i, load_spinor<R>(rows<R>(a.x + roff, 12, vh), i));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) bb.c[sp][c] = bb.c[sp][c] - cx.c[sp][c] + acc.c[sp][c];
    store_spinor<R>(out, i, bb);
  } else {  // M_PREP
    Spinor<R> bb = load_spinor<R>(rows<R>(a.b + roff, 12, vh), i);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) bb.c[sp][c] = bb.c[sp][c] + acc.c[sp][c];
    store_spinor<R>(out, i, bb);
  }
}

template <typename R, int MODE>
static hipError_t launch_mode(const HopArgs<R>& a, bool dagger, int nrhs, hipStream_t s) {
  dim3 grid(a.nblk, nrhs), block(HOP_BLOCK);
  if (dagger)
    hipLaunchKernelGGL((hop_kernel<R, MODE, true>), grid, block, 0, s, a);
  else
    hipLaunchKernelGGL((hop_kernel<R, MODE, false>), grid, block, 0, s, a);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_hop(const HopArgs<R>& a0, int mode, bool dagger, int nrhs, hipStream_t s) {
  HopArgs<R> a = a0;
  int nb = (a.g.Vh + HOP_BLOCK - 1) / HOP_BLOCK;
  a.nblk = (nb + 7) & ~7;
  switch (mode) {
    case M_HOP_CLINV: return launch_mode<R, M_HOP_CLINV>(a, dagger, nrhs, s);
    case M_RECON: return launch_mode<R, M_RECON>(a, dagger, nrhs, s);
    case M_APPLY: return launch_mode<R, M_APPLY>(a, dagger, nrhs, s);
    case M_RICH: return launch_mode<R, M_RICH>(a, dagger, nrhs, s);
    case M_RESID: return launch_mode<R, M_RESID>(a, dagger, nrhs, s);
    case M_PREP: return launch_mode<R, M_PREP>(a, dagger, nrhs, s);
  }
  return hipErrorInvalidValue;
}

template <typename R>
__global__ void __launch_bounds__(HOP_BLOCK) k_clover_only(Geo g, const pair<R>* __restrict__ clov,
                                                            const pair<R>* __restrict__ v, pair<R>* __restrict__ out) {
  const int vh = g.Vh;
  const int i = blockIdx.x * HOP_BLOCK + (int)threadIdx.x;
  if (i >= vh) return;
  const size_t roff = (size_t)blockIdx.y * 12 * (size_t)vh;
  store_spinor<R>(rows<R>(out + roff, 12, vh), i,
                  clover_mul<R>(rows<R>(clov, 36, vh), i, load_spinor<R>(rows<R>(v + roff, 12, vh), i)));
}

template <typename R>
hipError_t launch_clover_only(const Geo& g, int nrhs, const pair<R>* clov, const pair<R>* v, pair<R>* out,
                              hipStream_t s) {
  dim3 grid((g.Vh + HOP_BLOCK - 1) / HOP_BLOCK, nrhs);
  hipLaunchKernelGGL((k_clover_only<R>), grid, dim3(HOP_BLOCK), 0, s, g, clov, v, out);
  return hipGetLastError();
}

template hipError_t launch_clover_only<double>(const Geo&, int, const d2_t*, const d2_t*, d2_t*, hipStream_t);
template hipError_t launch_clover_only<float>(const Geo&, int, const f2_t*, const f2_t*, f2_t*, hipStream_t);

template hipError_t launch_hop<double>(const HopArgs<double>&, int, bool, int, hipStream_t);
template hipError_t launch_hop<float>(const HopArgs<float>&, int, bool, int, hipStream_t);

}  // namespace ddq
