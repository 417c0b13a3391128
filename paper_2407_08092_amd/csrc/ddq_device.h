// ddq_device.h -- device-side building blocks of the odd-even Wilson-clover kernels.
//
// Conventions are those of include/ddq.h: chiral gamma basis, hopping term
// H = 1/2 sum_mu [(1 - g_mu) U_mu(x) T_+mu + (1 + g_mu) U_mu(x-mu)^H T_-mu], clover
// blocks as two Hermitian 6x6 matrices per site (Sect. 2.4.5).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace ddq {

// ---------------------------------------------------------------------------
// complex arithmetic on (re, im) pairs
// ---------------------------------------------------------------------------
template <typename R> struct cpx { R r, i; };

// native two-element vectors: one 16-byte (FP64) or 8-byte (FP32) access per complex
typedef double d2_t __attribute__((ext_vector_type(2)));
typedef float f2_t __attribute__((ext_vector_type(2)));
template <typename R> struct pair_t;
template <> struct pair_t<double> { using type = d2_t; };
template <> struct pair_t<float> { using type = f2_t; };
template <typename R> using pair = typename pair_t<R>::type;

template <typename R> __device__ __forceinline__ cpx<R> mk(R r, R i) { return {r, i}; }
template <typename R> __device__ __forceinline__ cpx<R> operator+(cpx<R> a, cpx<R> b) { return {a.r + b.r, a.i + b.i}; }
template <typename R> __device__ __forceinline__ cpx<R> operator-(cpx<R> a, cpx<R> b) { return {a.r - b.r, a.i - b.i}; }
template <typename R> __device__ __forceinline__ cpx<R> operator*(cpx<R> a, cpx<R> b) {
  return {a.r * b.r - a.i * b.i, a.r * b.i + a.i * b.r};
}
template <typename R> __device__ __forceinline__ cpx<R> operator*(R s, cpx<R> a) { return {s * a.r, s * a.i}; }
template <typename R> __device__ __forceinline__ cpx<R> conj(cpx<R> a) { return {a.r, -a.i}; }
// conj(a) * b
template <typename R> __device__ __forceinline__ cpx<R> cmul_conj(cpx<R> a, cpx<R> b) {
  return {a.r * b.r + a.i * b.i, a.r * b.i - a.i * b.r};
}
template <typename R> __device__ __forceinline__ cpx<R> times_i(cpx<R> a) { return {-a.i, a.r}; }
template <typename R> __device__ __forceinline__ cpx<R> times_minus_i(cpx<R> a) { return {a.i, -a.r}; }
// acc += a * b
template <typename R> __device__ __forceinline__ void cfma(cpx<R>& acc, cpx<R> a, cpx<R> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(-a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(a.i, b.r, acc.i);
}
// acc += conj(a) * b
template <typename R> __device__ __forceinline__ void cfma_conj(cpx<R>& acc, cpx<R> a, cpx<R> b) {
  acc.r = fma(a.r, b.r, acc.r);
  acc.r = fma(a.i, b.i, acc.r);
  acc.i = fma(a.r, b.i, acc.i);
  acc.i = fma(-a.i, b.r, acc.i);
}

// Every field is stored as rows of 16-byte elements, one per site: an element holds
// CPE<R> complex numbers (one in FP64, two in FP32), so every load is a 16-byte
// access per lane.  Logical complex row r of a field lives in element row
// r / CPE, slot r % CPE.  Fields are read through raw buffer descriptors: the
// descriptor (base, byte size) lives in SGPRs, the element-row offset in the scalar
// soffset operand and the lane's site in one 32-bit VGPR offset, so a twelve-row
// spinor gather costs one VGPR of address.  Reads past the descriptor's size return
// zero instead of faulting.  Every offset stays below 4 GiB: a descriptor never
// spans more than one spinor, one link direction or one clover field.

// cache-policy bits of the streamed (read-once) link and clover loads: 2 = nt
// (non-temporal), which keeps them from evicting the neighbour spinor rows that
// eight sites reuse (measured +12% on the 48^3 x 96 stencil)
#ifndef DDQ_STREAM_AUX
#define DDQ_STREAM_AUX 2
#endif
// cache-policy bits of the spinor loads (reused by the eight neighbours)
#ifndef DDQ_SPINOR_AUX
#define DDQ_SPINOR_AUX 0
#endif

typedef unsigned int u2_t __attribute__((ext_vector_type(2)));
typedef unsigned int u4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
constexpr int BUF_DWORD3 = 0x00020000;  // gfx9-family raw buffer format word

// complex numbers per 16-byte element
template <typename R> struct cpe_t { static constexpr int value = 16 / (int)sizeof(pair<R>); };
template <typename R> constexpr int CPE = cpe_t<R>::value;

// complex rows of the three field kinds
constexpr int SPINOR_ROWS = 12;  // 4 spins x 3 colours
constexpr int LINK_ROWS = 18;    // per direction mu: U_mu(x) (9 entries), then U_mu(x - mu)^H (9)
constexpr int CLOVER_ROWS = 36;  // 2 blocks x 18 (re, im) slots

struct Field {
  __amdgpu_buffer_rsrc_t rsrc;
  uint32_t row_bytes;  // bytes between element rows
};

// parity vector: element rows of V/2 elements each
__device__ __forceinline__ Field vfield(const void* base, int erows, int vh) {
  Field f;
  const uint32_t rb = (uint32_t)vh * 16u;
  f.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)(rb * (uint32_t)erows), BUF_DWORD3);
  f.row_bytes = rb;
  return f;
}
__device__ __forceinline__ uint32_t voff(int i) { return (uint32_t)i * 16u; }

// Link and clover fields (read once per kernel) are stored in blocks of
// DDQ_FIELD_BLOCK sites: all element rows of one block are contiguous, so one
// wavefront's link (or clover) is a single contiguous run of memory.  0 selects
// plain rows.
#ifndef DDQ_FIELD_BLOCK
#define DDQ_FIELD_BLOCK 64
#endif
__host__ __device__ __forceinline__ int field_vh(int vh) {
  return DDQ_FIELD_BLOCK ? ((vh + DDQ_FIELD_BLOCK - 1) / DDQ_FIELD_BLOCK) * DDQ_FIELD_BLOCK : vh;
}
// element index of (element row, site i) in an erows-row blocked field
__host__ __device__ __forceinline__ size_t fidx(int row, int i, int erows, int vh) {
  if (DDQ_FIELD_BLOCK)
    return ((size_t)(i / DDQ_FIELD_BLOCK) * erows + row) * DDQ_FIELD_BLOCK + (i % DDQ_FIELD_BLOCK);
  return (size_t)row * vh + i;
}
__device__ __forceinline__ Field bfield(const void* base, int erows, int vh) {
  if (!DDQ_FIELD_BLOCK) return vfield(base, erows, vh);
  Field f;
  const uint32_t total = (uint32_t)field_vh(vh) * (uint32_t)erows * 16u;
  f.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)total, BUF_DWORD3);
  f.row_bytes = DDQ_FIELD_BLOCK * 16u;
  return f;
}
__device__ __forceinline__ uint32_t boff(int i, int erows) {
  if (!DDQ_FIELD_BLOCK) return voff(i);
  return (uint32_t)((i / DDQ_FIELD_BLOCK) * erows * DDQ_FIELD_BLOCK + (i % DDQ_FIELD_BLOCK)) * 16u;
}

template <int AUX = 0>
__device__ __forceinline__ u4_t ld16(const Field& f, int row, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(f.rsrc, (int)off, (int)(row * f.row_bytes), AUX);
}
// A vector store reads its data registers after it issues (the read is tracked by
// the EXP counter); the compiler may schedule a write to those registers before that
// read has happened, and the store then writes the new values.  Measured on gfx950:
// kernels that store one right-hand side and reuse the registers for the next
// returned nondeterministic wrong values, which an expcnt(0) wait after each store
// removes.  Every kernel whose stores are followed by more register writes calls
// store_fence() after them.
__device__ __forceinline__ void store_fence() {
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt(0xCF0F);  // expcnt(0); vmcnt and lgkmcnt left at their maxima
  __builtin_amdgcn_sched_barrier(0);
}
// cache-policy bits of the stencil's output stores: nt, so that written rows do not
// displace the neighbour rows still to be read (measured +3.7% on the 48^3 x 96 apply)
#ifndef DDQ_STORE_AUX
#define DDQ_STORE_AUX 2
#endif
// cache-policy bits of the epilogue's own-site loads (x, b: read once per launch): nt
#ifndef DDQ_OWN_AUX
#define DDQ_OWN_AUX 2
#endif
__device__ __forceinline__ void st16(const Field& f, int row, uint32_t off, u4_t v) {
  __builtin_amdgcn_raw_buffer_store_b128(v, f.rsrc, (int)off, (int)(row * f.row_bytes), DDQ_STORE_AUX);
  store_fence();
}

// 16-byte element <-> CPE complex numbers
template <typename R>
__device__ __forceinline__ void unpack(u4_t q, cpx<R>* c) {
  if constexpr (sizeof(R) == 8) {
    d2_t d = __builtin_bit_cast(d2_t, q);
    c[0] = {d.x, d.y};
  } else {
    f4_t f = __builtin_bit_cast(f4_t, q);
    c[0] = {f.x, f.y};
    c[1] = {f.z, f.w};
  }
}
template <typename R>
__device__ __forceinline__ u4_t pack(const cpx<R>* c) {
  if constexpr (sizeof(R) == 8) {
    d2_t d;
    d.x = c[0].r;
    d.y = c[0].i;
    return __builtin_bit_cast(u4_t, d);
  } else {
    f4_t f;
    f.x = c[0].r;
    f.y = c[0].i;
    f.z = c[1].r;
    f.w = c[1].i;
    return __builtin_bit_cast(u4_t, f);
  }
}

// complex rows [r0, r0 + n) of a field (n a multiple of CPE, r0 too)
template <typename R, int AUX = 0>
__device__ __forceinline__ void load_rows(const Field& f, int r0, int n, uint32_t off, cpx<R>* out) {
#pragma unroll
  for (int k = 0; k < n / CPE<R>; ++k) unpack<R>(ld16<AUX>(f, r0 / CPE<R> + k, off), out + k * CPE<R>);
}

// ---------------------------------------------------------------------------
// geometry of one parity: checkerboard index i <-> coordinates
// ---------------------------------------------------------------------------
struct Geo {
  int L[4];      // Lx, Ly, Lz, Lt
  int Lxh;       // Lx / 2
  int Vh;        // V / 2
  int sY, sZ, sT;  // checkerboard strides of y, z, t: Lxh, Lxh*Ly, Lxh*Ly*Lz
  int antiperiodic;
};

struct Site {
  int i, x, y, z, t;
};

// coordinates of checkerboard site i of parity p
__device__ __forceinline__ Site decode(const Geo& g, int i, int p) {
  Site s;
  s.i = i;
  int xh = i % g.Lxh;
  int r = i / g.Lxh;
  s.y = r % g.L[1];
  r /= g.L[1];
  s.z = r % g.L[2];
  s.t = r / g.L[2];
  s.x = 2 * xh + ((p + s.y + s.z + s.t) & 1);
  return s;
}

// XCD-aware workgroup order: the dispatcher deals workgroups round-robin over the
// eight XCDs; renumber them so that every XCD walks one contiguous range of sites
// and the neighbour reuse in y and z stays inside that XCD's L2.
// Renumbering workgroups so that each XCD walks one contiguous range measured
// slower on the 48^3 x 96 stencil (4.06 vs 4.71 TB/s): with the dispatcher's own
// round-robin order all XCDs work on neighbouring sites at once and share the
// neighbour rows through the Infinity Cache.  Kept as an option.
#ifndef DDQ_XCD_REMAP
#define DDQ_XCD_REMAP 0
#endif
// Chunked order: the dispatcher deals workgroups round-robin over the 8 XCDs;
// with DDQ_XCD_CHUNK = C each XCD instead receives C consecutive workgroups of
// every group of 8 C, so block-boundary neighbours share an L2.
#ifndef DDQ_XCD_CHUNK
#define DDQ_XCD_CHUNK 0
#endif
__device__ __forceinline__ int xcd_block(int nblocks_padded) {
  int b = blockIdx.x;
  if (DDQ_XCD_CHUNK > 0) {
    const int C = DDQ_XCD_CHUNK;
    const int grp = b / (8 * C), r = b % (8 * C);
    return grp * 8 * C + (r % 8) * C + r / 8;
  }
  if (!DDQ_XCD_REMAP) return b;
  int per = nblocks_padded >> 3;
  return (b & 7) * per + (b >> 3);
}

// Slab order.  Each t-slice (g.sT sites) is cut into eight contiguous pieces of whole
// 64-site groups; XCD k (workgroup w runs on XCD w mod 8) walks piece k of slice 0,
// then piece k of slice 1, and so on.  All XCDs advance through the same t-slices
// together, and the z- and t-neighbours of an XCD's sites lie in its own pieces a few
// workgroups apart, so they are fetched once into that XCD's L2.
// q: the caller's 64-site group within XCD xcd's walk.  Returns false past the end;
// else sets [base, end): the group's sites (end clips a partial group at the slice end).
__device__ __forceinline__ bool slab_group(const Geo& g, int xcd, int q, int& base, int& end) {
  const int P = g.sT;
  const int ng = (P + 63) >> 6;
  const int g0 = (xcd * ng) >> 3, n = (((xcd + 1) * ng) >> 3) - g0;
  if (n <= 0) return false;
  const int t = q / n;
  if (t >= g.L[3]) return false;
  base = t * P + (g0 + q - t * n) * 64;
  end = min(base + 64, (t + 1) * P);
  return true;
}
// 64-site groups in the longest XCD walk
inline long long slab_groups_per_xcd(const Geo& g) {
  const long long ng = (g.sT + 63) / 64;
  return (long long)g.L[3] * ((ng + 7) / 8);
}

// ---------------------------------------------------------------------------
// spinors: 4 spins x 3 colours
// ---------------------------------------------------------------------------
template <typename R> struct Spinor { cpx<R> c[4][3]; };
template <typename R> struct Half { cpx<R> c[2][3]; };

template <typename R> __device__ __forceinline__ void zero(Spinor<R>& s) {
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) s.c[a][b] = {R(0), R(0)};
}

// spinor of a parity vector (12 complex rows) at lane offset off = voff(i)
template <typename R, int AUX = DDQ_SPINOR_AUX>
__device__ __forceinline__ Spinor<R> load_spinor(const Field& v, uint32_t off) {
  cpx<R> c[SPINOR_ROWS];
  load_rows<R, AUX>(v, 0, SPINOR_ROWS, off, c);
  Spinor<R> s;
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) s.c[a][b] = c[3 * a + b];
  return s;
}
template <typename R>
__device__ __forceinline__ void store_spinor(const Field& v, uint32_t off, const Spinor<R>& s) {
  cpx<R> c[SPINOR_ROWS];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < 3; ++b) c[3 * a + b] = s.c[a][b];
#pragma unroll
  for (int k = 0; k < SPINOR_ROWS / CPE<R>; ++k) st16(v, k, off, pack<R>(c + k * CPE<R>));
}

// Spin projection (1 + sg * g_mu) psi in the chiral basis.  With
// g_mu = [[0, B], [B^H, 0]] (B_1 = -i s1, B_2 = -i s2, B_3 = -i s3, B_4 = 1) the
// projected spinor is (h, sg * B^H h) with h = psi_up + sg * B psi_dn, so only
// the two-spin h goes through the SU(3) multiply.
template <int MU, typename R>
__device__ __forceinline__ Half<R> project(const Spinor<R>& p, R sg) {
  Half<R> h;
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    cpx<R> b0, b1;  // B psi_dn
    if (MU == 0) {        // B = [[0, -i], [-i, 0]]
      b0 = times_minus_i(p.c[3][c]);
      b1 = times_minus_i(p.c[2][c]);
    } else if (MU == 1) { // B = [[0, -1], [1, 0]]
      b0 = {-p.c[3][c].r, -p.c[3][c].i};
      b1 = p.c[2][c];
    } else if (MU == 2) { // B = [[-i, 0], [0, i]]
      b0 = times_minus_i(p.c[2][c]);
      b1 = times_i(p.c[3][c]);
    } else {              // B = 1
      b0 = p.c[2][c];
      b1 = p.c[3][c];
    }
    h.c[0][c] = p.c[0][c] + sg * b0;
    h.c[1][c] = p.c[1][c] + sg * b1;
  }
  return h;
}

// acc += f * (h, sg * B^H h): reconstruct the lower spins of a projected spinor
template <int MU, typename R>
__device__ __forceinline__ void accumulate(Spinor<R>& acc, const Half<R>& h, R sg) {
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    acc.c[0][c] = acc.c[0][c] + h.c[0][c];
    acc.c[1][c] = acc.c[1][c] + h.c[1][c];
    cpx<R> d0, d1;  // B^H h
    if (MU == 0) {        // B^H = [[0, i], [i, 0]]
      d0 = times_i(h.c[1][c]);
      d1 = times_i(h.c[0][c]);
    } else if (MU == 1) { // B^H = [[0, 1], [-1, 0]]
      d0 = h.c[1][c];
      d1 = {-h.c[0][c].r, -h.c[0][c].i};
    } else if (MU == 2) { // B^H = [[i, 0], [0, -i]]
      d0 = times_i(h.c[0][c]);
      d1 = times_minus_i(h.c[1][c]);
    } else {
      d0 = h.c[0][c];
      d1 = h.c[1][c];
    }
    acc.c[2][c] = acc.c[2][c] + sg * d0;
    acc.c[3][c] = acc.c[3][c] + sg * d1;
  }
}


// a 3x3 link, 9 row-major entries
template <typename R> struct Link { cpx<R> u[9]; };

// one direction's link field: LINK_ROWS complex rows (U_mu(x), then U_mu(x - mu)^H)
template <typename R>
__device__ __forceinline__ Link<R> load_link_half(const Field& U, int half, uint32_t off) {
  Link<R> l;
  load_rows<R, DDQ_STREAM_AUX>(U, 9 * half, 9, off, l.u);  // FP64 only: 9 rows = 9 elements
  return l;
}
// SU(3) from its first two rows: row 2 = conj(row 0 x row 1)
template <typename R>
__device__ __forceinline__ void su3_third_row(Link<R>& l) {
  l.u[6] = conj(l.u[1] * l.u[5] - l.u[2] * l.u[4]);
  l.u[7] = conj(l.u[2] * l.u[3] - l.u[0] * l.u[5]);
  l.u[8] = conj(l.u[0] * l.u[4] - l.u[1] * l.u[3]);
}

// 12-real storage (LINK12_ROWS complex rows per direction: the first two rows of
// U_mu(x), then of U_mu(x - mu)^H); the third rows are rebuilt
constexpr int LINK12_ROWS = 12;
template <typename R>
__device__ __forceinline__ void load_link_pair12(const Field& U, uint32_t off, Link<R>& fwd, Link<R>& bwd) {
  cpx<R> c[LINK12_ROWS];
  load_rows<R, DDQ_STREAM_AUX>(U, 0, LINK12_ROWS, off, c);
#pragma unroll
  for (int e = 0; e < 6; ++e) {
    fwd.u[e] = c[e];
    bwd.u[e] = c[6 + e];
  }
  su3_third_row(fwd);  // the backward link's third row is rebuilt where it is used
}

template <typename R>
__device__ __forceinline__ void load_link_pair(const Field& U, uint32_t off, Link<R>& fwd, Link<R>& bwd) {
  cpx<R> c[LINK_ROWS];
  load_rows<R, DDQ_STREAM_AUX>(U, 0, LINK_ROWS, off, c);
#pragma unroll
  for (int e = 0; e < 9; ++e) {
    fwd.u[e] = c[e];
    bwd.u[e] = c[9 + e];
  }
}

// U h on both spins of a half spinor
template <typename R>
__device__ __forceinline__ Half<R> link_mul(const Link<R>& U, const Half<R>& h) {
  Half<R> o;
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      cpx<R> acc = U.u[3 * a] * h.c[s][0];
      cfma(acc, U.u[3 * a + 1], h.c[s][1]);
      cfma(acc, U.u[3 * a + 2], h.c[s][2]);
      o.c[s][a] = acc;
    }
  return o;
}

// ---------------------------------------------------------------------------
// clover blocks: Hermitian 6x6, 18 (re, im) slots per block:
//   slots 0..2  diagonal pairs (d0, d1), (d2, d3), (d4, d5)
//   slots 3..17 upper triangle a_jk, j < k, row-major ((0,1), (0,2), ..., (4,5))
// a site's clover field has CLOVER_ROWS = 36 complex rows: block 0 slots, then block 1.
// ---------------------------------------------------------------------------
__host__ __device__ constexpr int tri_slot(int j, int k) {  // j < k
  return 3 + j * 5 - (j * (j - 1)) / 2 + (k - j - 1);
}

template <typename R>
__device__ __forceinline__ void clover_block_apply(const cpx<R>* sl, const cpx<R> in[6], cpx<R> out[6]) {
  R d[6];
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    d[2 * k] = sl[k].r;
    d[2 * k + 1] = sl[k].i;
  }
#pragma unroll
  for (int j = 0; j < 6; ++j) out[j] = d[j] * in[j];
#pragma unroll
  for (int j = 0; j < 6; ++j)
#pragma unroll
    for (int k = j + 1; k < 6; ++k) {
      cpx<R> ajk = sl[tri_slot(j, k)];
      cfma(out[j], ajk, in[k]);
      cfma_conj(out[k], ajk, in[j]);
    }
}

// out = A psi for the two blocks of a site (block 0: spins 0,1; block 1: spins 2,3).
// C: the clover field (bfield, CLOVER_ROWS / CPE element rows); off = boff(i, ...)
template <typename R>
__device__ __forceinline__ Spinor<R> clover_mul(const Field& C, uint32_t off, const Spinor<R>& p) {
  Spinor<R> o;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    cpx<R> sl[18];
    load_rows<R, DDQ_STREAM_AUX>(C, 18 * b, 18, off, sl);
    cpx<R> in[6], out[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) in[k] = p.c[2 * b + k / 3][k % 3];
    clover_block_apply<R>(sl, in, out);
#pragma unroll
    for (int k = 0; k < 6; ++k) o.c[2 * b + k / 3][k % 3] = out[k];
  }
  return o;
}

}  // namespace ddq
