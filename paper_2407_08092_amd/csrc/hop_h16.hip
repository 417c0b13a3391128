// hop_h16.hip -- the Schur-complement stencil with 16-bit storage and FP32 arithmetic.
//
// Spinors, links and clover blocks are stored as IEEE half (FP16) or bfloat16
// values; every load is widened to FP32 and all arithmetic is FP32, so only the
// storage rounding differs from the FP32 path.  A 16-byte element holds four
// complex numbers:
//   spinor   12 complex rows -> 3 element rows (rows 4e..4e+3 in element e)
//   links    12-real only: per direction the first two rows of U_mu(x) and of
//            U_mu(x - mu)^H (12 complex rows, 3 element rows); third rows rebuilt
//   clover   each 6x6 block's 18 slots padded to 20 -> 10 element rows per site
// Per even site the Schur apply moves 944 bytes (FP32 with 12-real links: 1824).
// Link and clover fields use the blocked 64-site layout of the other paths.
#include "hop_common.h"

namespace ddq {

typedef unsigned short u16_t;

template <typename S>
__device__ __forceinline__ float h2f(u16_t b) {
  return (float)__builtin_bit_cast(S, b);
}
template <typename S>
__device__ __forceinline__ u16_t f2h(float f) {
  return __builtin_bit_cast(u16_t, (S)f);
}

// element <-> four complex numbers; complex j is word j (re: low half, im: high half)
template <typename S>
__device__ __forceinline__ void unpack4(u4_t q, cpx<float>* c) {
#pragma unroll
  for (int j = 0; j < 4; ++j) c[j] = {h2f<S>((u16_t)(q[j] & 0xffffu)), h2f<S>((u16_t)(q[j] >> 16))};
}
template <typename S>
__device__ __forceinline__ u4_t pack4(const cpx<float>* c) {
  u4_t q;
#pragma unroll
  for (int j = 0; j < 4; ++j) q[j] = (unsigned)f2h<S>(c[j].r) | ((unsigned)f2h<S>(c[j].i) << 16);
  return q;
}

constexpr int SP16_E = 3;   // element rows of a spinor
constexpr int LK16_E = 3;   // element rows of one direction's 12-real link pair
constexpr int CL16_E = 10;  // element rows of a site's clover (2 blocks x 5)

template <typename S>
__device__ __forceinline__ Spinor<float> unpack_spinor(const u4_t (&q)[SP16_E]) {
  cpx<float> c[12];
#pragma unroll
  for (int e = 0; e < SP16_E; ++e) unpack4<S>(q[e], c + 4 * e);
  Spinor<float> s;
#pragma unroll
  for (int k = 0; k < 12; ++k) s.c[k / 3][k % 3] = c[k];
  return s;
}
template <typename S, int AUX = DDQ_SPINOR_AUX>
__device__ __forceinline__ Spinor<float> load_spinor16(const Field& v, uint32_t off) {
  u4_t q[SP16_E];
#pragma unroll
  for (int e = 0; e < SP16_E; ++e) q[e] = ld16<AUX>(v, e, off);
  return unpack_spinor<S>(q);
}
template <typename S>
__device__ __forceinline__ void store_spinor16(const Field& v, uint32_t off, const Spinor<float>& s) {
  cpx<float> c[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) c[k] = s.c[k / 3][k % 3];
#pragma unroll
  for (int e = 0; e < SP16_E; ++e) st16(v, e, off, pack4<S>(c + 4 * e));
}

// raw loads of one hop for nb right-hand sides, issued one hop ahead of their use
template <int NB>
struct Raw16 {
  u4_t sp[NB][SP16_E];
  u4_t lk[LK16_E];
};

struct Ctx16 {
  HopCtx<float> h;  // neighbours, projector signs
  const u4_t* links;
  int vh;
  uint32_t loff;
};

template <int H, int NB>
__device__ __forceinline__ void load_raw(const Ctx16& c, const Field (&in)[NB], Raw16<NB>& r) {
#pragma unroll
  for (int q = 0; q < NB; ++q)
#pragma unroll
    for (int e = 0; e < SP16_E; ++e) r.sp[q][e] = ld16<DDQ_SPINOR_AUX>(in[q], e, voff(c.h.nb.j[H]));
  if constexpr ((H & 1) == 0) {
    const Field lf = bfield(c.links + (size_t)(H >> 1) * LK16_E * field_vh(c.vh), LK16_E, c.vh);
#pragma unroll
    for (int e = 0; e < LK16_E; ++e) r.lk[e] = ld16<DDQ_STREAM_AUX>(lf, e, c.loff);
  }
}

template <int H, typename S, int NB>
__device__ __forceinline__ void compute16(Spinor<float> (&acc)[NB], const Raw16<NB>& r, Link<float>& ub,
                                          const Ctx16& c) {
  Link<float> u;
  if constexpr ((H & 1) == 0) {
    cpx<float> l[12];
#pragma unroll
    for (int e = 0; e < LK16_E; ++e) unpack4<S>(r.lk[e], l + 4 * e);
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      u.u[k] = l[k];
      ub.u[k] = l[6 + k];
    }
  } else {
    u = ub;
  }
  su3_third_row(u);
#pragma unroll
  for (int q = 0; q < NB; ++q) hop_compute<H, float>(acc[q], unpack_spinor<S>(r.sp[q]), u, c.h);
}

template <int H, typename S, int NB>
__device__ __forceinline__ void steps16(Spinor<float> (&acc)[NB], const Raw16<NB>& cur, Link<float>& ub,
                                        const Ctx16& c, const Field (&in)[NB]) {
  if constexpr (H < 7) {
    Raw16<NB> nxt;
    load_raw<H + 1, NB>(c, in, nxt);
    compute16<H, S, NB>(acc, cur, ub, c);
#pragma unroll
    for (int q = 0; q < NB; ++q) hop_fence<float>(acc[q]);
    steps16<H + 1, S, NB>(acc, nxt, ub, c, in);
  } else {
    compute16<H, S, NB>(acc, cur, ub, c);
#pragma unroll
    for (int q = 0; q < NB; ++q) hop_fence<float>(acc[q]);
  }
}

// the 18 slots of clover block b (element rows 5b..5b+4; the last two slots pad)
template <typename S>
__device__ __forceinline__ void clover_slots16(const Field& C, uint32_t off, int b, cpx<float> (&sl)[20]) {
#pragma unroll
  for (int e = 0; e < 5; ++e) unpack4<S>(ld16<DDQ_STREAM_AUX>(C, 5 * b + e, off), sl + 4 * e);
}

// spinor rows of clover block b (spins 2b, 2b+1: rows 6b..6b+5)
__device__ __forceinline__ void block_rows(const Spinor<float>& s, int b, cpx<float> out[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) out[k] = s.c[2 * b + k / 3][k % 3];
}
__device__ __forceinline__ void set_block_rows(Spinor<float>& s, int b, const cpx<float> in[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) s.c[2 * b + k / 3][k % 3] = in[k];
}

// One thread per output site and NB right-hand sides; workgroup blk covers 256 sites
// of one group of NB right-hand sides (tile_site); the links and clover slots of the
// site are loaded once for the NB spinors.
// C32: the clover blocks come from the FP32 field (CLOVER_ROWS complex rows, two per
// 16-byte element) instead of the 16-bit one
template <typename S, int MODE, int NB, bool C32>
__global__ void __launch_bounds__(HOP_BLOCK) __attribute__((amdgpu_waves_per_eu(NB > 1 ? 2 : 4)))
hop16_kernel(Hop16Args a) {
  const int vh = a.g.Vh;
  int i, rg;
  if (!tile_site(a.g, (int)blockIdx.x, a.nrhs / NB, a.chunk, HOP_BLOCK, (int)threadIdx.x, i, rg)) return;
  const int r0 = rg * NB;
  Field in[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) in[q] = vfield(a.in + (size_t)(r0 + q) * SP16_E * (size_t)vh, SP16_E, vh);
  Ctx16 c;
  c.links = a.links;
  c.vh = vh;
  c.loff = boff(i, LK16_E);
  c.h.nb = neighbours(a.g, decode(a.g, i, a.p_out));
  c.h.sf = -1.f;  // D: forward (1 - g), backward (1 + g)
  c.h.sb = 1.f;

  Spinor<float> acc[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) zero(acc[q]);
  {
    Raw16<NB> r;
    Link<float> ub;
    load_raw<0, NB>(c, in, r);
    steps16<0, S, NB>(acc, r, ub, c, in);
  }

  constexpr int CL_E = C32 ? CLOVER_ROWS / CPE<float> : CL16_E;
  const Field cl = bfield(C32 ? (const void*)a.clov32 : (const void*)a.clov, CL_E, vh);
  const uint32_t coff = boff(i, CL_E);
  const uint32_t off = voff(i);
  auto slots = [&](int b, cpx<float>(&sl)[20]) {
    if constexpr (C32)
      load_rows<float, DDQ_STREAM_AUX>(cl, 18 * b, 18, coff, sl);
    else
      clover_slots16<S>(cl, coff, b, sl);
  };
  // epilogue: per right-hand side, both clover blocks (their slots loaded once
  // for the NB spinors; with one right-hand side, block by block)
  cpx<float> sl[2][20];
  if constexpr (NB > 1) {
    slots(0, sl[0]);
    slots(1, sl[1]);
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const size_t roff = (size_t)(r0 + q) * SP16_E * (size_t)vh;
    Spinor<float> xx, bb;
    if constexpr (MODE != M_HOP_CLINV) xx = load_spinor16<S, DDQ_OWN_AUX>(vfield(a.x + roff, SP16_E, vh), off);
    if constexpr (MODE == M_RICH) bb = load_spinor16<S, DDQ_OWN_AUX>(vfield(a.b + roff, SP16_E, vh), off);
    Spinor<float> res;
#pragma unroll
    for (int b = 0; b < 2; ++b) {
      if constexpr (NB == 1) slots(b, sl[b]);
      cpx<float> h[6], o[6];
      block_rows(acc[q], b, h);
#pragma unroll
      for (int k = 0; k < 6; ++k) h[k] = 0.5f * h[k];
      if constexpr (MODE == M_HOP_CLINV) {
        clover_block_apply<float>(sl[b], h, o);
      } else {
        cpx<float> x6[6];
        block_rows(xx, b, x6);
        clover_block_apply<float>(sl[b], x6, o);
        if constexpr (MODE == M_APPLY) {
#pragma unroll
          for (int k = 0; k < 6; ++k) o[k] = o[k] - h[k];
        } else {  // M_RICH
          cpx<float> b6[6];
          block_rows(bb, b, b6);
#pragma unroll
          for (int k = 0; k < 6; ++k) o[k] = x6[k] + a.omega * (b6[k] - o[k] + h[k]);
        }
      }
      set_block_rows(res, b, o);
    }
    store_spinor16<S>(vfield(a.out + roff, SP16_E, vh), off, res);  // may alias a.x (in place)
  }
}

template <typename S, int NB, bool C32>
static hipError_t launch16_c(const Hop16Args& a, int mode, dim3 grid, dim3 block, hipStream_t s) {
  switch (mode) {
    case M_HOP_CLINV: hipLaunchKernelGGL((hop16_kernel<S, M_HOP_CLINV, NB, C32>), grid, block, 0, s, a); break;
    case M_APPLY: hipLaunchKernelGGL((hop16_kernel<S, M_APPLY, NB, C32>), grid, block, 0, s, a); break;
    case M_RICH: hipLaunchKernelGGL((hop16_kernel<S, M_RICH, NB, C32>), grid, block, 0, s, a); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename S, int NB>
static hipError_t launch16_nb(const Hop16Args& a, int mode, hipStream_t s) {
  const long long nb = tile_grid_sites(a.g, HOP_BLOCK, a.nrhs / NB, a.chunk);
  if (nb > 0x7fffffffLL) return hipErrorInvalidValue;
  dim3 grid((unsigned)nb), block(HOP_BLOCK);
  return a.clov32 ? launch16_c<S, NB, true>(a, mode, grid, block, s) : launch16_c<S, NB, false>(a, mode, grid, block, s);
}

template <typename S>
static hipError_t launch16_s(const Hop16Args& a, int mode, hipStream_t s) {
  switch (a.nb) {
    case 1: return launch16_nb<S, 1>(a, mode, s);
    case 2: return launch16_nb<S, 2>(a, mode, s);
    case 3: return launch16_nb<S, 3>(a, mode, s);
  }
  return hipErrorInvalidValue;
}

hipError_t launch_hop16(int kind, const Hop16Args& a0, int mode, hipStream_t s) {
  Hop16Args a = a0;
  if (a.nb == 0)  // right-hand sides per thread: the largest of 3, 2, 1 dividing nrhs
    for (int nb = 3; nb >= 1; --nb)
      if (a.nrhs % nb == 0) {
        a.nb = nb;
        break;
      }
  if (a.nrhs < 1 || a.nb < 1 || a.nb > 3 || a.nrhs % a.nb != 0 || a.chunk < XMAP_SLAB || a.chunk > 1024)
    return hipErrorInvalidValue;
  return kind == H16_BF16 ? launch16_s<__bf16>(a, mode, s) : launch16_s<_Float16>(a, mode, s);
}

// ---------------------------------------------------------------------------
// conversions
// ---------------------------------------------------------------------------

// FP64 parity vectors [nrhs][12][vh] -> 16-bit [nrhs][3][vh] elements, times scale
template <typename S>
__global__ void k_parity_to_h16(u4_t* __restrict__ y, const d2_t* __restrict__ x, double scale, long long n3,
                                int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // (rhs, e, i)
  if (t >= n3) return;
  const int i = (int)(t % vh);
  const long long re = t / vh;
  const long long rhs = re / SP16_E;
  const int e = (int)(re % SP16_E);
  const d2_t* xr = x + rhs * 12LL * vh;
  cpx<float> c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    d2_t v = xr[(size_t)(4 * e + j) * vh + i];
    c[j] = {(float)(v.x * scale), (float)(v.y * scale)};
  }
  y[t] = pack4<S>(c);
}

template <typename S>
__global__ void k_parity_from_h16(d2_t* __restrict__ y, const u4_t* __restrict__ x, double scale, long long n3,
                                  int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n3) return;
  const int i = (int)(t % vh);
  const long long re = t / vh;
  const long long rhs = re / SP16_E;
  const int e = (int)(re % SP16_E);
  d2_t* yr = y + rhs * 12LL * vh;
  cpx<float> c[4];
  unpack4<S>(x[t], c);
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    d2_t v;
    v.x = (double)c[j].r * scale;
    v.y = (double)c[j].i * scale;
    yr[(size_t)(4 * e + j) * vh + i] = v;
    store_fence();
  }
}

// 16-bit [nrhs][3][vh] -> FP32 paired [nrhs][6][vh] (rows 2m, 2m+1), times scale
template <typename S>
__global__ void k_h16_to_f32(f4_t* __restrict__ y, const u4_t* __restrict__ x, float scale, long long n3, int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n3) return;
  const int i = (int)(t % vh);
  const long long re = t / vh;
  const long long rhs = re / SP16_E;
  const int e = (int)(re % SP16_E);
  cpx<float> c[4];
  unpack4<S>(x[t], c);
  f4_t* yr = y + rhs * 6LL * vh;
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    f4_t o;
    o.x = c[2 * h].r * scale;
    o.y = c[2 * h].i * scale;
    o.z = c[2 * h + 1].r * scale;
    o.w = c[2 * h + 1].i * scale;
    yr[(size_t)(2 * e + h) * vh + i] = o;
    store_fence();
  }
}

// FP64 blocked link fields of one parity (4 directions x LINK_ROWS) -> 16-bit
// 12-real (4 directions x LK16_E element rows)
template <typename S>
__global__ void k_links_to_h16(const d2_t* __restrict__ in, u4_t* __restrict__ out, int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= 4LL * LK16_E * vh) return;
  const int i = (int)(t % vh);
  const int e = (int)((t / vh) % LK16_E);
  const int mu = (int)(t / ((long long)vh * LK16_E));
  const size_t fv = (size_t)field_vh(vh);
  const d2_t* src = in + (size_t)mu * LINK_ROWS * fv;
  cpx<float> c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int k = 4 * e + j;             // 12-real row
    const int row = k < 6 ? k : k + 3;   // its row among the 18 stored entries
    d2_t v = src[fidx(row, i, LINK_ROWS, vh)];
    c[j] = {(float)v.x, (float)v.y};
  }
  out[(size_t)mu * LK16_E * fv + fidx(e, i, LK16_E, vh)] = pack4<S>(c);
}

// FP64 blocked clover field (CLOVER_ROWS) -> 16-bit (CL16_E element rows, each
// block's 18 slots padded to 20)
template <typename S>
__global__ void k_clover_to_h16(const d2_t* __restrict__ in, u4_t* __restrict__ out, int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)CL16_E * vh) return;
  const int i = (int)(t % vh);
  const int e = (int)(t / vh);
  const int b = e / 5, m = e % 5;
  cpx<float> c[4];
#pragma unroll
  for (int j = 0; j < 4; ++j) {
    const int slot = 4 * m + j;
    if (slot < 18) {
      d2_t v = in[fidx(18 * b + slot, i, CLOVER_ROWS, vh)];
      c[j] = {(float)v.x, (float)v.y};
    } else {
      c[j] = {0.f, 0.f};
    }
  }
  out[fidx(e, i, CL16_E, vh)] = pack4<S>(c);
}

#define DDQ_H16_GRID(n) dim3((unsigned)(((n) + 255) / 256)), dim3(256)

hipError_t launch_parity_to_h16(int kind, void* y, const d2_t* x, double scale, int nrhs, int vh, hipStream_t s) {
  const long long n3 = (long long)SP16_E * vh * nrhs;
  if (kind == H16_BF16)
    hipLaunchKernelGGL(k_parity_to_h16<__bf16>, DDQ_H16_GRID(n3), 0, s, (u4_t*)y, x, scale, n3, vh);
  else
    hipLaunchKernelGGL(k_parity_to_h16<_Float16>, DDQ_H16_GRID(n3), 0, s, (u4_t*)y, x, scale, n3, vh);
  return hipGetLastError();
}

hipError_t launch_parity_from_h16(int kind, d2_t* y, const void* x, double scale, int nrhs, int vh, hipStream_t s) {
  const long long n3 = (long long)SP16_E * vh * nrhs;
  if (kind == H16_BF16)
    hipLaunchKernelGGL(k_parity_from_h16<__bf16>, DDQ_H16_GRID(n3), 0, s, y, (const u4_t*)x, scale, n3, vh);
  else
    hipLaunchKernelGGL(k_parity_from_h16<_Float16>, DDQ_H16_GRID(n3), 0, s, y, (const u4_t*)x, scale, n3, vh);
  return hipGetLastError();
}

hipError_t launch_h16_to_f32(int kind, void* y, const void* x, float scale, int nrhs, int vh, hipStream_t s) {
  const long long n3 = (long long)SP16_E * vh * nrhs;
  if (kind == H16_BF16)
    hipLaunchKernelGGL(k_h16_to_f32<__bf16>, DDQ_H16_GRID(n3), 0, s, (f4_t*)y, (const u4_t*)x, scale, n3, vh);
  else
    hipLaunchKernelGGL(k_h16_to_f32<_Float16>, DDQ_H16_GRID(n3), 0, s, (f4_t*)y, (const u4_t*)x, scale, n3, vh);
  return hipGetLastError();
}

hipError_t launch_links_to_h16(int kind, const d2_t* in, void* out, int vh, hipStream_t s) {
  const long long n = 4LL * LK16_E * vh;
  if (kind == H16_BF16)
    hipLaunchKernelGGL(k_links_to_h16<__bf16>, DDQ_H16_GRID(n), 0, s, in, (u4_t*)out, vh);
  else
    hipLaunchKernelGGL(k_links_to_h16<_Float16>, DDQ_H16_GRID(n), 0, s, in, (u4_t*)out, vh);
  return hipGetLastError();
}

hipError_t launch_clover_to_h16(int kind, const d2_t* in, void* out, int vh, hipStream_t s) {
  const long long n = (long long)CL16_E * vh;
  if (kind == H16_BF16)
    hipLaunchKernelGGL(k_clover_to_h16<__bf16>, DDQ_H16_GRID(n), 0, s, in, (u4_t*)out, vh);
  else
    hipLaunchKernelGGL(k_clover_to_h16<_Float16>, DDQ_H16_GRID(n), 0, s, in, (u4_t*)out, vh);
  return hipGetLastError();
}

}  // namespace ddq
