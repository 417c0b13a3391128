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

// neighbour sites of hop h (h = 2 mu + 0: forward x + mu, h = 2 mu + 1: backward
// x - mu) and the boundary sign of the t hops
struct Nbr {
  int j[8];
  float sgn_tf, sgn_tb;
};

__device__ __forceinline__ Nbr neighbours(const Geo& g, const Site& s) {
  Nbr n;
  {
    int base = s.i - (s.x >> 1);
    int xf = (s.x + 1 == g.L[0]) ? 0 : s.x + 1;
    int xb = (s.x == 0) ? g.L[0] - 1 : s.x - 1;
    n.j[0] = base + (xf >> 1);
    n.j[1] = base + (xb >> 1);
  }
  n.j[2] = (s.y + 1 == g.L[1]) ? s.i - (g.L[1] - 1) * g.sY : s.i + g.sY;
  n.j[3] = (s.y == 0) ? s.i + (g.L[1] - 1) * g.sY : s.i - g.sY;
  n.j[4] = (s.z + 1 == g.L[2]) ? s.i - (g.L[2] - 1) * g.sZ : s.i + g.sZ;
  n.j[5] = (s.z == 0) ? s.i + (g.L[2] - 1) * g.sZ : s.i - g.sZ;
  const bool wf = (s.t + 1 == g.L[3]), wb = (s.t == 0);
  n.j[6] = wf ? s.i - (g.L[3] - 1) * g.sT : s.i + g.sT;
  n.j[7] = wb ? s.i + (g.L[3] - 1) * g.sT : s.i - g.sT;
  n.sgn_tf = (g.antiperiodic && wf) ? -1.f : 1.f;
  n.sgn_tb = (g.antiperiodic && wb) ? -1.f : 1.f;
  return n;
}

template <typename R>
__device__ __forceinline__ void scale_half(Half<R>& h, R f) {
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) h.c[s][c] = f * h.c[s][c];
}

// Orders one hop before the next: the accumulator is routed through an empty
// volatile asm, so the hop's arithmetic has to finish here, and the memory
// clobber keeps later loads below.  Without it the instruction selector lifts
// all 96 neighbour loads to the top and spills them.
template <typename R>
__device__ __forceinline__ void hop_fence(Spinor<R>& acc) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) asm volatile("" : "+v"(acc.c[sp][c].r), "+v"(acc.c[sp][c].i)::"memory");
  __builtin_amdgcn_sched_barrier(0);
}

// software pipelining: issue hop h+1's loads before hop h's arithmetic
#ifndef DDQ_PREFETCH
#define DDQ_PREFETCH 1
#endif

template <typename R>
struct HopCtx {
  Rows<R> in;
  const pair<R>* links;
  int vh;
  uint32_t loff;  // lane offset of the output site in a 9-row link field
  Nbr nb;
  R sf, sb;      // projector signs of forward and backward hops
};

template <int H, typename R>
__device__ __forceinline__ Link<R> hop_link(const HopCtx<R>& c) {
  // dirs 0..3: U_mu(x); dirs 4..7: U_mu(x - mu)^H
  constexpr int dir = (H & 1) ? 4 + (H >> 1) : (H >> 1);
  return load_link<R>(frows<R>(c.links + (size_t)dir * 9 * field_vh(c.vh), 9, c.vh), c.loff);
}

// acc += (1 + sg g_mu) U in(neighbour), hop H
template <int H, typename R>
__device__ __forceinline__ void hop_compute(Spinor<R>& acc, const Spinor<R>& p, const Link<R>& u,
                                            const HopCtx<R>& c) {
  constexpr int MU = H >> 1;
  const R sg = (H & 1) ? c.sb : c.sf;
  Half<R> h = project<MU, R>(p, sg);
  Half<R> uh = link_mul<R>(u, h);
  if (MU == 3) scale_half(uh, (R)((H & 1) ? c.nb.sgn_tb : c.nb.sgn_tf));
  accumulate<MU, R>(acc, uh, sg);
}

template <int H, typename R>
__device__ __forceinline__ void hop_steps(Spinor<R>& acc, Spinor<R>& p, Link<R>& u, const HopCtx<R>& c) {
  if constexpr (DDQ_PREFETCH && H < 7) {
    Spinor<R> pn = load_spinor<R>(c.in, c.nb.j[H + 1]);
    Link<R> un = hop_link<H + 1, R>(c);
    hop_compute<H, R>(acc, p, u, c);
    hop_fence<R>(acc);
    hop_steps<H + 1, R>(acc, pn, un, c);
  } else {
    hop_compute<H, R>(acc, p, u, c);
    hop_fence<R>(acc);
    if constexpr (H < 7) {
      Spinor<R> pn = load_spinor<R>(c.in, c.nb.j[H + 1]);
      Link<R> un = hop_link<H + 1, R>(c);
      hop_steps<H + 1, R>(acc, pn, un, c);
    }
  }
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
  const Rows<R> cl = frows<R>(a.clov, 36, vh);
  const uint32_t coff = foff<R>(i, 36);
  const Site s = decode(a.g, i, a.p_out);
  HopCtx<R> c;
  c.in = rows<R>(a.in + roff, 12, vh);
  c.links = a.links;
  c.vh = vh;
  c.loff = foff<R>(i, 9);
  c.nb = neighbours(a.g, s);
  // D: forward (1 - g), backward (1 + g).  D^H = g5 D g5 flips both projectors.
  c.sf = DAG ? R(1) : R(-1);
  c.sb = -c.sf;

  Spinor<R> acc;
  zero(acc);
  {
    Spinor<R> p = load_spinor<R>(c.in, c.nb.j[0]);
    Link<R> u = hop_link<0, R>(c);
    hop_steps<0, R>(acc, p, u, c);
  }
  // h = 1/2 acc
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.c[sp][c] = R(0.5) * acc.c[sp][c];

  const Rows<R> out = rows<R>(a.out + roff, 12, vh);  // may alias a.x (in-place Richardson)
  if constexpr (MODE == M_HOP_CLINV) {
    store_spinor<R>(out, i, clover_mul<R>(cl, coff, acc));
  } else if constexpr (MODE == M_RECON) {
    Spinor<R> bb = load_spinor<R>(rows<R>(a.b + roff, 12, vh), i);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) bb.c[sp][c] = bb.c[sp][c] + acc.c[sp][c];
    store_spinor<R>(out, i, clover_mul<R>(cl, coff, bb));
  } else if constexpr (MODE == M_APPLY) {
    Spinor<R> cx = clover_mul<R>(cl, coff, load_spinor<R>(rows<R>(a.x + roff, 12, vh), i));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int c = 0; c < 3; ++c) cx.c[sp][c] = cx.c[sp][c] - acc.c[sp][c];
    store_spinor<R>(out, i, cx);
  } else if constexpr (MODE == M_RICH) {
    Spinor<R> xx = load_spinor<R>(rows<R>(a.x + roff, 12, vh), i);
    Spinor<R> bb = load_spinor<R>(rows<R>(a.b + roff, 12, vh), i);
    Spinor<R> cx = clover_mul<R>(cl, coff, xx);
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
    Spinor<R> cx = clover_mul<R>(cl, coff, load_spinor<R>(rows<R>(a.x + roff, 12, vh), i));
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
  const int pad = 8 * (DDQ_XCD_CHUNK > 0 ? DDQ_XCD_CHUNK : 1);
  a.nblk = ((nb + pad - 1) / pad) * pad;
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
                  clover_mul<R>(frows<R>(clov, 36, vh), foff<R>(i, 36), load_spinor<R>(rows<R>(v + roff, 12, vh), i)));
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
