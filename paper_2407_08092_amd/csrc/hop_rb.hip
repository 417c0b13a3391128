// hop_rb.hip -- register-blocked FP32 stencil for several right-hand sides.
//
// The same operator as hop.hip (kernel A with its A_oo^-1 epilogue, kernel B as
// the Schur apply or a Richardson sweep), for nrhs right-hand sides that share the
// links and the clover field.  One thread computes one site for nb right-hand
// sides: the eight incident links and the clover slots are loaded once and
// applied to nb spinors, so their loads (and their bytes, were they not cached)
// are divided by nb, while every right-hand side still reads its own neighbour
// spinors.  The tile (nb, wavefronts per site block, XCD placement) is a launch
// parameter chosen per lattice and right-hand-side count by timing (ddq_tune).
#include "hop_common.h"

namespace ddq {

#ifndef DDQ_WAVES_RB
#define DDQ_WAVES_RB 2
#endif

// hop H for nb spinors: one link load (forward hops load the direction's pair and
// keep the backward link for hop H + 1), nb neighbour spinor loads
template <int H, bool L12, int NB>
__device__ __forceinline__ void rb_hops(Spinor<float> (&acc)[NB], Link<float>& ub, const HopCtx<float>& c,
                                        const Field (&in)[NB]) {
  using R = float;
  Link<R> u;
  if constexpr ((H & 1) == 0) {
    if constexpr (L12)
      load_link_pair12<R>(link_field(c, H >> 1), c.loff, u, ub);
    else
      load_link_pair<R>(link_field(c, H >> 1), c.loff, u, ub);
  } else {
    u = ub;
    if constexpr (L12) su3_third_row(u);
  }
  Spinor<R> p[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) p[q] = load_spinor<R>(in[q], voff(c.nb.j[H]));
#pragma unroll
  for (int q = 0; q < NB; ++q) hop_compute<H, R>(acc[q], p[q], u, c);
#pragma unroll
  for (int q = 0; q < NB; ++q) hop_fence<R>(acc[q]);
  if constexpr (H < 7) rb_hops<H + 1, L12, NB>(acc, ub, c, in);
}

// rows of clover block b of a spinor (spins 2b, 2b+1): complex rows 6b..6b+5,
// element rows 3b..3b+2
__device__ __forceinline__ void block_of(const Spinor<float>& s, int b, cpx<float> out[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = s.c[2 * b + k / 3][k % 3];
}
__device__ __forceinline__ void store_block(const Field& v, int b, uint32_t off, const cpx<float> c[6]) {
#pragma unroll
  for (int k = 0; k < 3; ++k) st16(v, 3 * b + k, off, pack<float>(c + 2 * k));
}

template <int MODE, bool L12, int NB, int G>
__global__ void __launch_bounds__(HOP_BLOCK) __attribute__((amdgpu_waves_per_eu(DDQ_WAVES_RB)))
hop_kernel_rb(HopArgs<float> a) {
  using R = float;
  constexpr int SPW = HOP_BLOCK / G;  // sites of a workgroup
  constexpr int SP_E = SPINOR_ROWS / CPE<R>;
  const int vh = a.g.Vh;
  const int GR = (a.nrhs + NB * G - 1) / (NB * G);  // workgroups per site block
  const int lane = G == 1 ? (int)threadIdx.x : ((int)threadIdx.x & 63);
  const int w = G == 1 ? 0 : __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  int i, rg;  // the dispatcher deals workgroups round-robin over 8 XCDs
  if (!tile_site(a.g, (int)blockIdx.x, GR, a.tile.xmap, SPW, lane, i, rg)) return;
  const int r0 = (rg * G + w) * NB;
  if (r0 >= a.nrhs) return;

  Field in[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) in[q] = vfield(a.in + (size_t)(r0 + q) * (size_t)a.rhs_stride, SP_E, vh);
  HopCtx<R> c;
  c.in = in[0];
  c.links = a.links;
  c.lrows = L12 ? LINK12_ROWS : LINK_ROWS;
  c.vh = vh;
  c.loff = boff(i, c.lrows / CPE<R>);
  c.nb = neighbours(a.g, decode(a.g, i, a.p_out));
  c.sf = R(-1);  // D: forward (1 - g), backward (1 + g)
  c.sb = R(1);

  Spinor<R> acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) zero(acc[q]);
  {
    Link<R> ub;
    rb_hops<0, L12, NB>(acc, ub, c, in);
  }

  // epilogue per clover block: its 18 slots are loaded once for the nb spinors
  const Field cl = bfield(a.clov, CLOVER_ROWS / CPE<R>, vh);
  const uint32_t coff = boff(i, CLOVER_ROWS / CPE<R>);
  const uint32_t off = voff(i);
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    cpx<R> sl[18];
    load_rows<R, DDQ_STREAM_AUX>(cl, 18 * b, 18, coff, sl);
#pragma unroll
    for (int q = 0; q < NB; ++q) {
      const size_t roff = (size_t)(r0 + q) * (size_t)a.rhs_stride;
      const Field out = vfield(a.out + roff, SP_E, vh);  // may alias a.x (in-place Richardson)
      cpx<R> h[6], o[6];
      block_of(acc[q], b, h);
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = R(0.5) * h[k];
      if constexpr (MODE == M_HOP_CLINV) {
        clover_block_apply<R>(sl, h, o);
      } else {
        cpx<R> xx[6];
        load_rows<R, DDQ_OWN_AUX>(vfield(a.x + roff, SP_E, vh), 6 * b, 6, off, xx);
        clover_block_apply<R>(sl, xx, o);
        if constexpr (MODE == M_APPLY) {
#pragma unroll
          for (int k = 0; k < 6; ++k) o[k] = o[k] - h[k];
        } else {  // M_RICH
          cpx<R> bb[6];
          load_rows<R, DDQ_OWN_AUX>(vfield(a.b + roff, SP_E, vh), 6 * b, 6, off, bb);
#pragma unroll
          for (int k = 0; k < 6; ++k) o[k] = xx[k] + a.omega * (bb[k] - o[k] + h[k]);
        }
      }
      store_block(out, b, off, o);
    }
  }
}

bool hop_rb_supported(int mode, bool dagger, int nrhs, const MrTile& t) {
  if (dagger || nrhs < 2) return false;
  if (mode != M_HOP_CLINV && mode != M_APPLY && mode != M_RICH) return false;
  if (t.passes < 1 || nrhs % t.passes != 0 || t.lds_kb < 0 || t.lds_kb > 160) return false;
  if (t.nb < 1 || t.nb > MR_MAX_NB || (nrhs / t.passes) % t.nb != 0) return false;
  if (t.xmap < XMAP_SLAB || t.xmap > 1024) return false;
  return t.g == 1 || t.g == 4;
}

template <int MODE, bool L12, int NB>
static hipError_t rb_launch_g(const HopArgs<float>& a, hipStream_t s) {
  const int G = a.tile.g;
  const int gr = (a.nrhs + NB * G - 1) / (NB * G);
  const long long nb = tile_grid_sites(a.g, HOP_BLOCK / G, gr, a.tile.xmap);
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  const unsigned lds = (unsigned)a.tile.lds_kb * 1024u;  // occupancy cap only: the kernel uses no LDS
  if (G == 1)
    hipLaunchKernelGGL((hop_kernel_rb<MODE, L12, NB, 1>), dim3((unsigned)nb), dim3(HOP_BLOCK), lds, s, a);
  else
    hipLaunchKernelGGL((hop_kernel_rb<MODE, L12, NB, 4>), dim3((unsigned)nb), dim3(HOP_BLOCK), lds, s, a);
  return hipGetLastError();
}

template <int MODE, bool L12>
static hipError_t rb_launch_nb(const HopArgs<float>& a, hipStream_t s) {
  switch (a.tile.nb) {
    case 1: return rb_launch_g<MODE, L12, 1>(a, s);
    case 2: return rb_launch_g<MODE, L12, 2>(a, s);
    case 3: return rb_launch_g<MODE, L12, 3>(a, s);
    case 4: return rb_launch_g<MODE, L12, 4>(a, s);
  }
  return hipErrorInvalidValue;
}

template <int MODE>
static hipError_t rb_launch_mode(const HopArgs<float>& a, hipStream_t s) {
  return a.link12 ? rb_launch_nb<MODE, true>(a, s) : rb_launch_nb<MODE, false>(a, s);
}

hipError_t launch_hop_rb(const HopArgs<float>& a0, int mode, int nrhs, hipStream_t s) {
  if (!hop_rb_supported(mode, false, nrhs, a0.tile)) return hipErrorInvalidValue;
  const int per = nrhs / a0.tile.passes;
  for (int p = 0; p < a0.tile.passes; ++p) {
    // pass p: right-hand sides [p per, (p + 1) per), every vector offset alike
    HopArgs<float> a = a0;
    const size_t off = (size_t)p * per * (size_t)a0.rhs_stride;
    a.in = a0.in + off;
    a.out = a0.out + off;
    if (a0.x) a.x = a0.x + off;
    if (a0.b) a.b = a0.b + off;
    a.nrhs = per;
    hipError_t e = hipErrorInvalidValue;
    switch (mode) {
      case M_HOP_CLINV: e = rb_launch_mode<M_HOP_CLINV>(a, s); break;
      case M_APPLY: e = rb_launch_mode<M_APPLY>(a, s); break;
      case M_RICH: e = rb_launch_mode<M_RICH>(a, s); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace ddq
