// hop.hip -- the stencil kernels of the Schur complement D_S = A_ee - H_eo A_oo^-1 H_oe
// (eq. 3 with D_eo = -H_eo, D_oe = -H_oe, D_ee = A_ee, D_oo = A_oo).
//
// One thread per output site.  All fields are structure-of-arrays per parity
// (row stride V/2), so every load of a neighbour row, a link entry or a clover
// slot is one coalesced 8- or 16-byte access per lane.  Each site carries its
// eight incident links (forward U_mu(x) and pre-daggered backward U_mu(x-mu)^H),
// so link reads never gather.  Kernel A (odd output) and kernel B (even output)
// are one template with different epilogues (HopMode).
#include "hop_common.h"

namespace ddq {

// register budget: waves per SIMD the scheduler must keep resident.  FP32 with 12-real
// links asks for 3: under the budget of 4 those kernels spill 8 bytes a lane, under that of 3
// they are scheduled into 127 registers without spills and still run 4 waves per SIMD.
#ifndef DDQ_WAVES_F64
#define DDQ_WAVES_F64 2
#endif
#ifndef DDQ_WAVES_F32
#define DDQ_WAVES_F32 4
#endif
#ifndef DDQ_WAVES_F32_L12
#define DDQ_WAVES_F32_L12 3
#endif
// workgroup order of the one-right-hand-side kernels: 0 = the dispatcher's, 1 = slab
// order (slab_group)
#ifndef DDQ_SITE_ORDER
#define DDQ_SITE_ORDER 1
#endif
template <typename R, bool L12> struct HOP_WAVES {
  static constexpr int value = L12 ? DDQ_WAVES_F32_L12 : DDQ_WAVES_F32;
};
template <bool L12> struct HOP_WAVES<double, L12> { static constexpr int value = DDQ_WAVES_F64; };

// site of this thread in a one-right-hand-side launch (grid: one_rhs_grid); false if none.
// t_cnt > 0 restricts the launch to the output sites of slices [t_lo, t_lo + t_cnt).
__device__ __forceinline__ bool one_rhs_site(const Geo& g, int nblk, int& i, int t_lo = 0, int t_cnt = 0) {
#if DDQ_SITE_ORDER
  int q = (int)(blockIdx.x >> 3) * (HOP_BLOCK / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  if (t_cnt > 0) {
    const int ng = (g.sT + 63) >> 6, xcd = (int)(blockIdx.x & 7);
    const int n = (((xcd + 1) * ng) >> 3) - ((xcd * ng) >> 3);  // this XCD's groups per slice
    if (n <= 0 || q >= t_cnt * n) return false;
    q += t_lo * n;
  }
  int base, end;
  if (!slab_group(g, (int)(blockIdx.x & 7), q, base, end)) return false;
  i = base + ((int)threadIdx.x & 63);
  return i < end;
#else
  i = xcd_block(nblk) * HOP_BLOCK + (int)threadIdx.x;
  return i < g.Vh;
#endif
}
static int one_rhs_grid(const Geo& g, int t_cnt = 0) {
#if DDQ_SITE_ORDER
  const long long groups = t_cnt > 0 ? (long long)t_cnt * (((g.sT + 63) / 64 + 7) / 8) : slab_groups_per_xcd(g);
  const long long per = (groups + HOP_BLOCK / 64 - 1) / (HOP_BLOCK / 64);
  return 8 * per > 0x7fffffffLL ? -1 : (int)(8 * per);
#else
  int nb = (g.Vh + HOP_BLOCK - 1) / HOP_BLOCK;
  const int pad = 8 * (DDQ_XCD_CHUNK > 0 ? DDQ_XCD_CHUNK : 1);
  return ((nb + pad - 1) / pad) * pad;
#endif
}

template <typename R, int MODE, bool DAG, bool L12, bool MR>
__global__ void __launch_bounds__(HOP_BLOCK) __attribute__((amdgpu_waves_per_eu(HOP_WAVES<R, L12>::value)))
hop_kernel(HopArgs<R> a) {
  const int vh = a.g.Vh;
  int i, rhs;
  if constexpr (!MR) {
    if (!one_rhs_site(a.g, a.nblk, i, a.t_lo, a.t_cnt)) return;
    rhs = 0;
  } else {
    // several right-hand sides: a workgroup is 64 sites x (HOP_BLOCK / 64) right-hand
    // sides, so its wavefronts read the same link and clover entries; the workgroups
    // of the other right-hand-side groups of the same 64 sites follow it on the same
    // XCD (workgroup order a.tile.xmap, tile_site)
    // the wavefront's right-hand side, made explicitly uniform (an SGPR)
    const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
    const int groups = (a.nrhs + HOP_BLOCK / 64 - 1) / (HOP_BLOCK / 64);
    int rg;
    if (!tile_site(a.g, (int)blockIdx.x, groups, a.tile.xmap, 64, (int)threadIdx.x & 63, i, rg)) return;
    rhs = rg * (HOP_BLOCK / 64) + w;
    if (rhs >= a.nrhs) return;
  }
  if (i >= vh) return;
  constexpr int SP_E = SPINOR_ROWS / CPE<R>;  // element rows of a spinor
  const size_t roff = (size_t)rhs * (size_t)a.rhs_stride;
  const Field cl = bfield(a.clov, CLOVER_ROWS / CPE<R>, vh);
  const uint32_t coff = boff(i, CLOVER_ROWS / CPE<R>);
  const uint32_t off = voff(i);
  const Site s = decode(a.g, i, a.p_out);
  HopCtx<R> c;
  c.in = vfield(a.in + roff, SP_E, vh);
  c.links = a.links;
  c.lrows = L12 ? LINK12_ROWS : LINK_ROWS;
  c.vh = vh;
  c.loff = boff(i, c.lrows / CPE<R>);
  c.nb = neighbours(a.g, s);
  // D: forward (1 - g), backward (1 + g).  D^H = g5 D g5 flips both projectors.
  c.sf = DAG ? R(1) : R(-1);
  c.sb = -c.sf;

  Spinor<R> acc;
  zero(acc);
  {
    Spinor<R> p;
    Link<R> u, ub;
    hop_loads<0, R, L12>(c, p, u, ub);
    hop_steps<0, R, L12>(acc, p, u, ub, c);
  }
  // h = 1/2 acc
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc.c[sp][cc] = R(0.5) * acc.c[sp][cc];

  const Field out = vfield(a.out + roff, SP_E, vh);  // may alias a.x (in-place Richardson)
  if constexpr (MODE == M_HOP_CLINV) {
    store_spinor<R>(out, off, clover_mul<R>(cl, coff, acc));
  } else if constexpr (MODE == M_RECON) {
    Spinor<R> bb = load_spinor<R, DDQ_OWN_AUX>(vfield(a.b + roff, SP_E, vh), off);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) bb.c[sp][cc] = bb.c[sp][cc] + acc.c[sp][cc];
    store_spinor<R>(out, off, clover_mul<R>(cl, coff, bb));
  } else if constexpr (MODE == M_APPLY) {
    Spinor<R> cx = clover_mul<R>(cl, coff, load_spinor<R, DDQ_OWN_AUX>(vfield(a.x + roff, SP_E, vh), off));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) cx.c[sp][cc] = cx.c[sp][cc] - acc.c[sp][cc];
    store_spinor<R>(out, off, cx);
  } else if constexpr (MODE == M_RICH) {
    Spinor<R> xx = load_spinor<R, DDQ_OWN_AUX>(vfield(a.x + roff, SP_E, vh), off);
    Spinor<R> bb = load_spinor<R, DDQ_OWN_AUX>(vfield(a.b + roff, SP_E, vh), off);
    Spinor<R> cx = clover_mul<R>(cl, coff, xx);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        cpx<R> r = bb.c[sp][cc] - cx.c[sp][cc] + acc.c[sp][cc];
        xx.c[sp][cc] = xx.c[sp][cc] + a.omega * r;
      }
    store_spinor<R>(out, off, xx);
  } else if constexpr (MODE == M_RESID) {
    Spinor<R> bb = load_spinor<R, DDQ_OWN_AUX>(vfield(a.b + roff, SP_E, vh), off);
    Spinor<R> cx = clover_mul<R>(cl, coff, load_spinor<R, DDQ_OWN_AUX>(vfield(a.x + roff, SP_E, vh), off));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) bb.c[sp][cc] = bb.c[sp][cc] - cx.c[sp][cc] + acc.c[sp][cc];
    store_spinor<R>(out, off, bb);
  } else {  // M_PREP
    Spinor<R> bb = load_spinor<R, DDQ_OWN_AUX>(vfield(a.b + roff, SP_E, vh), off);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) bb.c[sp][cc] = bb.c[sp][cc] + acc.c[sp][cc];
    store_spinor<R>(out, off, bb);
  }
}

// Streaming ceiling of hop_kernel<R, MODE> with one right-hand side (a measurement
// aid, not part of D_S): every site moves the element rows the stencil kernel moves
// once per site -- the input spinor (the site's own rows in place of its eight
// neighbours'), the four link fields, the clover field, x and b where the mode reads
// them, the output rows -- with the same layouts, workgroup order and cache
// policies, combined by XOR without arithmetic.
// sites per thread of the streaming probe: with 2, a wavefront streams two consecutive
// 64-site groups (an experiment on run lengths; the stencil kernels use one)
#ifndef DDQ_STREAM_SPL
#define DDQ_STREAM_SPL 1
#endif
template <typename R, int MODE, bool L12>
__device__ __forceinline__ void stream_site(const HopArgs<R>& a, int i);

template <typename R, int MODE, bool L12>
__global__ void __launch_bounds__(HOP_BLOCK) hop_stream_kernel(HopArgs<R> a) {
#if DDQ_STREAM_SPL == 2
  const int q = (int)(blockIdx.x >> 3) * (HOP_BLOCK / 64) + __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int base0, end0, base1, end1;
  const bool ok0 = slab_group(a.g, (int)(blockIdx.x & 7), 2 * q, base0, end0);
  const bool ok1 = slab_group(a.g, (int)(blockIdx.x & 7), 2 * q + 1, base1, end1);
  const int i0 = base0 + ((int)threadIdx.x & 63), i1 = base1 + ((int)threadIdx.x & 63);
  if (ok0 && i0 < end0) stream_site<R, MODE, L12>(a, i0);
  if (ok1 && i1 < end1) stream_site<R, MODE, L12>(a, i1);
}
#else
  int i;
  if (!one_rhs_site(a.g, a.nblk, i)) return;
  stream_site<R, MODE, L12>(a, i);
}
#endif

template <typename R, int MODE, bool L12>
__device__ __forceinline__ void stream_site(const HopArgs<R>& a, int i) {
  const int vh = a.g.Vh;
  constexpr int SP_E = SPINOR_ROWS / CPE<R>;
  constexpr int LR = L12 ? LINK12_ROWS : LINK_ROWS;
  constexpr int CL_E = CLOVER_ROWS / CPE<R>;
  const uint32_t off = voff(i);
  u4_t acc = {0u, 0u, 0u, 0u};
  const Field in = vfield(a.in, SP_E, vh);
#pragma unroll
  for (int k = 0; k < SP_E; ++k) acc ^= ld16<DDQ_SPINOR_AUX>(in, k, off);
  const uint32_t loff = boff(i, LR / CPE<R>);
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const Field U = bfield(a.links + (size_t)mu * LR * field_vh(vh), LR / CPE<R>, vh);
#pragma unroll
    for (int k = 0; k < LR / CPE<R>; ++k) acc ^= ld16<DDQ_STREAM_AUX>(U, k, loff);
  }
  const Field cl = bfield(a.clov, CL_E, vh);
  const uint32_t coff = boff(i, CL_E);
#pragma unroll
  for (int k = 0; k < CL_E; ++k) acc ^= ld16<DDQ_STREAM_AUX>(cl, k, coff);
  if constexpr (MODE != M_HOP_CLINV) {
    const Field x = vfield(a.x, SP_E, vh);
#pragma unroll
    for (int k = 0; k < SP_E; ++k) acc ^= ld16<DDQ_OWN_AUX>(x, k, off);
  }
  if constexpr (MODE == M_RICH) {
    const Field b = vfield(a.b, SP_E, vh);
#pragma unroll
    for (int k = 0; k < SP_E; ++k) acc ^= ld16<DDQ_OWN_AUX>(b, k, off);
  }
  const Field out = vfield(a.out, SP_E, vh);
#pragma unroll
  for (int k = 0; k < SP_E; ++k) {
    u4_t v = acc;
    v.x += (unsigned)k;
    st16(out, k, off, v);
  }
}

template <typename R>
hipError_t launch_hop_stream(const HopArgs<R>& a0, int mode, hipStream_t s) {
  HopArgs<R> a = a0;
  a.nblk = one_rhs_grid(a.g);
  if (a.nblk < 0) return hipErrorInvalidValue;
  const bool l12 = sizeof(R) == 4 && a.link12;
  constexpr bool F32 = sizeof(R) == 4;
  dim3 grid(DDQ_STREAM_SPL == 2 ? ((a.nblk / 8 + 1) / 2) * 8 : a.nblk), block(HOP_BLOCK);
#define DDQ_STREAM_LAUNCH(M)                                                    \
  if (l12)                                                                      \
    hipLaunchKernelGGL((hop_stream_kernel<R, M, F32>), grid, block, 0, s, a);   \
  else                                                                          \
    hipLaunchKernelGGL((hop_stream_kernel<R, M, false>), grid, block, 0, s, a)
  switch (mode) {
    case M_HOP_CLINV: DDQ_STREAM_LAUNCH(M_HOP_CLINV); break;
    case M_APPLY: DDQ_STREAM_LAUNCH(M_APPLY); break;
    case M_RICH: DDQ_STREAM_LAUNCH(M_RICH); break;
    default: return hipErrorInvalidValue;
  }
#undef DDQ_STREAM_LAUNCH
  return hipGetLastError();
}
template hipError_t launch_hop_stream<float>(const HopArgs<float>&, int, hipStream_t);
template hipError_t launch_hop_stream<double>(const HopArgs<double>&, int, hipStream_t);

template <typename R, int MODE>
static hipError_t launch_mode(const HopArgs<R>& a, bool dagger, int nrhs, hipStream_t s) {
  dim3 block(HOP_BLOCK), grid(a.nblk);
  if (nrhs > 1) {
    const int groups = (nrhs + HOP_BLOCK / 64 - 1) / (HOP_BLOCK / 64);
    if (a.tile.xmap < XMAP_SLAB || a.tile.xmap > 1024) return hipErrorInvalidValue;
    const long long nb = tile_grid_sites(a.g, 64, groups, a.tile.xmap);
    if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
    grid = dim3((unsigned)nb);
  }
  // 12-real links exist for FP32 storage only
  const bool l12 = sizeof(R) == 4 && a.link12;
  constexpr bool F32 = sizeof(R) == 4;
#define DDQ_HOP_LAUNCH(D, L, M) hipLaunchKernelGGL((hop_kernel<R, MODE, D, L, M>), grid, block, 0, s, a)
  if (nrhs > 1) {
    if (l12) {
      if (dagger) DDQ_HOP_LAUNCH(true, F32, true); else DDQ_HOP_LAUNCH(false, F32, true);
    } else {
      if (dagger) DDQ_HOP_LAUNCH(true, false, true); else DDQ_HOP_LAUNCH(false, false, true);
    }
  } else {
    if (l12) {
      if (dagger) DDQ_HOP_LAUNCH(true, F32, false); else DDQ_HOP_LAUNCH(false, F32, false);
    } else {
      if (dagger) DDQ_HOP_LAUNCH(true, false, false); else DDQ_HOP_LAUNCH(false, false, false);
    }
  }
#undef DDQ_HOP_LAUNCH
  return hipGetLastError();
}

template <typename R>
hipError_t launch_hop(const HopArgs<R>& a0, int mode, bool dagger, int nrhs, hipStream_t s) {
  HopArgs<R> a = a0;
  a.nrhs = nrhs;
  if (a.t_cnt < 0 || a.t_lo < 0 || a.t_lo + a.t_cnt > a.g.L[3] || (a.t_cnt > 0 && nrhs != 1))
    return hipErrorInvalidValue;
  a.nblk = one_rhs_grid(a.g, a.t_cnt);
  if (a.nblk < 0) return hipErrorInvalidValue;
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
  constexpr int SP_E = SPINOR_ROWS / CPE<R>;
  store_spinor<R>(vfield(out + roff, SP_E, vh), voff(i),
                  clover_mul<R>(bfield(clov, CLOVER_ROWS / CPE<R>, vh), boff(i, CLOVER_ROWS / CPE<R>),
                                load_spinor<R>(vfield(v + roff, SP_E, vh), voff(i))));
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
