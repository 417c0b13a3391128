// hop_mrhs.hip -- FP32 stencil for several right-hand sides stored site-major with the
// right-hand sides interleaved ("mrhs" layout).
//
// The operator is that of hop.hip (kernel A with its A_oo^-1 epilogue, kernel B as the
// Schur apply or a Richardson sweep; eq. 3), applied to nrhs vectors that share the
// links and the clover blocks.  Layout of a parity vector: 16-byte element (i, k, r) =
// rows 2k, 2k+1 (k = 0..5) of right-hand side r at checkerboard site i, at element
// index (6 i + k) nrhs + r, so all right-hand sides of a site are one contiguous run
// of 96 nrhs bytes.
//
// A lane computes one (site, right-hand side): `lps` consecutive lanes (a multiple of
// four) share a site, so a wavefront covers 64 / lps sites and every neighbour gather
// of a wavefront reads whole runs.  Compared with one site per lane, a wavefront has a
// few sites in flight instead of 64, which keeps the rows that eight neighbours reuse
// inside an XCD's L2 between their uses.  The lanes of a site load the same link and
// clover entries (one request per cache line).
//
// The SU(3) products of a hop -- U (3 x 3) times the two projected spins of every
// right-hand side -- run either on the vector units or on the matrix cores with
// v_mfma_f32_4x4x1_16b_f32: each 4-lane block of a site is one of the instruction's
// sixteen 4 x 4 outer-product blocks, lane 4b + a supplies row a of the link (row 3:
// zero) as the A operand and its own projected spinor entry as the B operand, and lane
// 4b + j receives rows 0..2 of column j, i.e. its own right-hand side's product; four
// real instructions per complex colour term (Re += Ur hr - Ui hi, Im += Ur hi + Ui hr).
#include "hop_common.h"

#include <algorithm>

namespace ddq {

// register budget (waves per SIMD): the vector-unit form keeps whole links in registers
#ifndef DDQ_WAVES_MRHS_VALU
#define DDQ_WAVES_MRHS_VALU 3
#endif
#ifndef DDQ_WAVES_MRHS_MFMA
#define DDQ_WAVES_MRHS_MFMA 4
#endif
#ifndef DDQ_WAVES_MRHS_MFMA_TW
#define DDQ_WAVES_MRHS_MFMA_TW 3
#endif

// element row k of this layout sits nrhs elements after row k - 1 (the Field's
// row_bytes), a site's rows 6 nrhs elements after the previous site's
__device__ __forceinline__ Field mrhs_field(const void* base, int nrhs, int vh) {
  Field f;
  const uint32_t total = (uint32_t)vh * 6u * (uint32_t)nrhs * 16u;
  f.rsrc = __builtin_amdgcn_make_buffer_rsrc((void*)base, (short)0, (int)total, BUF_DWORD3);
  f.row_bytes = (uint32_t)nrhs * 16u;
  return f;
}
__device__ __forceinline__ uint32_t mrhs_off(int i, int r, int nrhs) {
  return ((uint32_t)i * 6u * (uint32_t)nrhs + (uint32_t)r) * 16u;
}

// slab order (slab_group) for groups of gs sites
__device__ __forceinline__ bool slab_group_n(const Geo& g, int xcd, int q, int gs, int& base, int& end) {
  const int P = g.sT;
  const int ng = (P + gs - 1) / gs;
  const int g0 = (xcd * ng) >> 3, n = (((xcd + 1) * ng) >> 3) - g0;
  if (n <= 0) return false;
  const int t = q / n;
  if (t >= g.L[3]) return false;
  base = t * P + (g0 + q - t * n) * gs;
  end = min(base + gs, (t + 1) * P);
  return true;
}

// the link data of one direction that a lane keeps: the whole forward and backward
// links (vector units) or the lane's row of each (matrix cores)
template <bool MF> struct LinkPairT;
template <> struct LinkPairT<false> { Link<float> f, b; };
template <> struct LinkPairT<true> { cpx<float> f[3], b[3]; };

template <bool MF, bool L12>
__device__ __forceinline__ void load_pair(const HopCtx<float>& c, int mu, int row, LinkPairT<MF>& lp) {
  const Field U = link_field(c, mu);
  if constexpr (!MF) {
    if constexpr (L12)
      load_link_pair12<float>(U, c.loff, lp.f, lp.b);
    else
      load_link_pair<float>(U, c.loff, lp.f, lp.b);
  } else if constexpr (L12) {
    // rows 0, 1 of both links are stored; the lane takes its row, rebuilding row 2
    Link<float> f, b;
    load_link_pair12<float>(U, c.loff, f, b);
    su3_third_row(b);
    const int a = row > 2 ? 2 : row;
    const float z = row > 2 ? 0.f : 1.f;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      cpx<float> fv = a == 0 ? f.u[e] : (a == 1 ? f.u[3 + e] : f.u[6 + e]);
      cpx<float> bv = a == 0 ? b.u[e] : (a == 1 ? b.u[3 + e] : b.u[6 + e]);
      lp.f[e] = z * fv;
      lp.b[e] = z * bv;
    }
  } else {
    // 18-real field: entries 0..8 forward, 9..17 backward, two per 16-byte element;
    // row a covers entries 3a..3a+2 and 9+3a..11+3a, i.e. elements f0, f0+1 and b0, b0+1
    const int a = row > 2 ? 2 : row;
    const int f0 = a == 0 ? 0 : (a == 1 ? 1 : 3);
    const int b0 = a == 0 ? 4 : (a == 1 ? 6 : 7);
    const uint32_t rb = U.row_bytes;
    cpx<float> F0[2], F1[2], B0[2], B1[2];
    unpack<float>(__builtin_amdgcn_raw_buffer_load_b128(U.rsrc, (int)(c.loff + (uint32_t)f0 * rb), 0, DDQ_STREAM_AUX), F0);
    unpack<float>(__builtin_amdgcn_raw_buffer_load_b128(U.rsrc, (int)(c.loff + (uint32_t)(f0 + 1) * rb), 0, DDQ_STREAM_AUX), F1);
    unpack<float>(__builtin_amdgcn_raw_buffer_load_b128(U.rsrc, (int)(c.loff + (uint32_t)b0 * rb), 0, DDQ_STREAM_AUX), B0);
    unpack<float>(__builtin_amdgcn_raw_buffer_load_b128(U.rsrc, (int)(c.loff + (uint32_t)(b0 + 1) * rb), 0, DDQ_STREAM_AUX), B1);
    const bool fo = a == 1;  // forward row starts in the odd slot of its first element
    const bool bo = a != 1;  // backward row likewise
    const float z = row > 2 ? 0.f : 1.f;
    lp.f[0] = z * (fo ? F0[1] : F0[0]);
    lp.f[1] = z * (fo ? F1[0] : F0[1]);
    lp.f[2] = z * (fo ? F1[1] : F1[0]);
    lp.b[0] = z * (bo ? B0[1] : B0[0]);
    lp.b[1] = z * (bo ? B1[0] : B0[1]);
    lp.b[2] = z * (bo ? B1[1] : B1[0]);
  }
}

// ---------------------------------------------------------------------------
// LDS staging of a site's links and clover slots.  The lps lanes of a site need the same
// 36 link elements (4 directions x 9, 16 bytes each; 6 a direction when 12-real) and 18
// clover elements; without staging every lane loads all of them (one vector-memory
// instruction per element for the whole wavefront).  Staged, lane rl of the site loads
// elements rl, rl + lps, ... once into the wavefront's LDS slot of the site, and the
// lanes read what they need from LDS.
// ---------------------------------------------------------------------------
constexpr int ST_LINK_E = 9;             // element stride of one direction in a slot
constexpr int ST_CLOV = 4 * ST_LINK_E;   // first clover element of a slot
constexpr int ST_SITE_E = ST_CLOV + 18;  // elements of a slot

// 16-byte load of element row e (per lane) of field f at lane offset off
__device__ __forceinline__ u4_t ld16_row(const Field& f, int e, uint32_t off) {
  return __builtin_amdgcn_raw_buffer_load_b128(f.rsrc, (int)(off + (uint32_t)e * f.row_bytes), 0, DDQ_STREAM_AUX);
}

// LDS slots of a wavefront: one per lane group (ceil(64 / lps) of them)
__device__ __forceinline__ int stage_slots(int lps) { return (64 + lps - 1) / lps; }

// order the wavefront's LDS accesses around the staging: every lane's writes before any
// lane's reads (and the reads of the previous site before the next site's writes)
__device__ __forceinline__ void wave_lds_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

template <bool L12>
__device__ __forceinline__ void stage_site(const HopCtx<float>& c, const Field& cl, uint32_t coff, int rl, int lps,
                                           u4_t* st) {
  constexpr int LE = (L12 ? LINK12_ROWS : LINK_ROWS) / 2;  // elements of one direction
  wave_lds_sync();
#pragma unroll
  for (int mu = 0; mu < 4; ++mu) {
    const Field U = link_field(c, mu);
    for (int e0 = 0; e0 < LE; e0 += lps) {
      const int e = e0 + rl;
      if (e < LE) st[mu * ST_LINK_E + e] = ld16_row(U, e, c.loff);
    }
  }
  for (int e0 = 0; e0 < 18; e0 += lps) {
    const int e = e0 + rl;
    if (e < 18) st[ST_CLOV + e] = ld16_row(cl, e, coff);
  }
  wave_lds_sync();
}

// load_pair from the staged slot
template <bool MF, bool L12>
__device__ __forceinline__ void load_pair_st(const u4_t* st, int mu, int row, LinkPairT<MF>& lp) {
  const u4_t* d = st + mu * ST_LINK_E;
  if constexpr (!MF) {
    cpx<float> c[18];
    constexpr int LE = (L12 ? LINK12_ROWS : LINK_ROWS) / 2;
#pragma unroll
    for (int e = 0; e < LE; ++e) unpack<float>(d[e], c + 2 * e);
    if constexpr (L12) {
#pragma unroll
      for (int e = 0; e < 6; ++e) {
        lp.f.u[e] = c[e];
        lp.b.u[e] = c[6 + e];
      }
      su3_third_row(lp.f);  // the backward link's third row is rebuilt at its hop
    } else {
#pragma unroll
      for (int e = 0; e < 9; ++e) {
        lp.f.u[e] = c[e];
        lp.b.u[e] = c[9 + e];
      }
    }
  } else if constexpr (L12) {
    Link<float> f, b;
    cpx<float> c[12];
#pragma unroll
    for (int e = 0; e < 6; ++e) unpack<float>(d[e], c + 2 * e);
#pragma unroll
    for (int e = 0; e < 6; ++e) {
      f.u[e] = c[e];
      b.u[e] = c[6 + e];
    }
    su3_third_row(f);
    su3_third_row(b);
    const int a = row > 2 ? 2 : row;
    const float z = row > 2 ? 0.f : 1.f;
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      lp.f[e] = z * (a == 0 ? f.u[e] : (a == 1 ? f.u[3 + e] : f.u[6 + e]));
      lp.b[e] = z * (a == 0 ? b.u[e] : (a == 1 ? b.u[3 + e] : b.u[6 + e]));
    }
  } else {
    const int a = row > 2 ? 2 : row;
    const int f0 = a == 0 ? 0 : (a == 1 ? 1 : 3);
    const int b0 = a == 0 ? 4 : (a == 1 ? 6 : 7);
    cpx<float> F0[2], F1[2], B0[2], B1[2];
    unpack<float>(d[f0], F0);
    unpack<float>(d[f0 + 1], F1);
    unpack<float>(d[b0], B0);
    unpack<float>(d[b0 + 1], B1);
    const bool fo = a == 1, bo = a != 1;
    const float z = row > 2 ? 0.f : 1.f;
    lp.f[0] = z * (fo ? F0[1] : F0[0]);
    lp.f[1] = z * (fo ? F1[0] : F0[1]);
    lp.f[2] = z * (fo ? F1[1] : F1[0]);
    lp.b[0] = z * (bo ? B0[1] : B0[0]);
    lp.b[1] = z * (bo ? B1[0] : B0[1]);
    lp.b[2] = z * (bo ? B1[1] : B1[0]);
  }
}

// out = A psi with the clover slots of the staged slot
__device__ __forceinline__ Spinor<float> clover_mul_st(const u4_t* st, const Spinor<float>& p) {
  Spinor<float> o;
#pragma unroll
  for (int b = 0; b < 2; ++b) {
    cpx<float> sl[18];
#pragma unroll
    for (int e = 0; e < 9; ++e) unpack<float>(st[ST_CLOV + 9 * b + e], sl + 2 * e);
    cpx<float> in[6], out[6];
#pragma unroll
    for (int k = 0; k < 6; ++k) in[k] = p.c[2 * b + k / 3][k % 3];
    clover_block_apply<float>(sl, in, out);
#pragma unroll
    for (int k = 0; k < 6; ++k) o.c[2 * b + k / 3][k % 3] = out[k];
  }
  return o;
}

// uh[s][.] = U h[s][.] for both projected spins on the matrix cores; urow: this lane's
// row of U (zero for row 3)
__device__ __forceinline__ Half<float> link_mul_mfma(const cpx<float> urow[3], const Half<float>& h) {
  Half<float> o;
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    f4_t dr = {0.f, 0.f, 0.f, 0.f}, di = {0.f, 0.f, 0.f, 0.f};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      dr = __builtin_amdgcn_mfma_f32_4x4x1f32(urow[c].r, h.c[s][c].r, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_4x4x1f32(urow[c].r, h.c[s][c].i, di, 0, 0, 0);
      dr = __builtin_amdgcn_mfma_f32_4x4x1f32(urow[c].i, -h.c[s][c].i, dr, 0, 0, 0);
      di = __builtin_amdgcn_mfma_f32_4x4x1f32(urow[c].i, h.c[s][c].r, di, 0, 0, 0);
    }
    o.c[s][0] = {dr[0], di[0]};
    o.c[s][1] = {dr[1], di[1]};
    o.c[s][2] = {dr[2], di[2]};
  }
  return o;
}

template <int H, bool MF, bool L12>
__device__ __forceinline__ void mrhs_hop(Spinor<float>& acc, const Spinor<float>& p, const LinkPairT<MF>& lp,
                                         const HopCtx<float>& c) {
  using R = float;
  if constexpr (!MF) {
    Link<R> u = (H & 1) ? lp.b : lp.f;
    if constexpr (L12 && (H & 1)) su3_third_row(u);
    hop_compute<H, R>(acc, p, u, c);
  } else {
    constexpr int MU = H >> 1;
    const R sg = (H & 1) ? c.sb : c.sf;
    Half<R> h = project<MU, R>(p, sg);
    if (MU == 3) scale_half(h, (R)((H & 1) ? c.nb.sgn_tb : c.nb.sgn_tf));
    Half<R> uh = link_mul_mfma((H & 1) ? lp.b : lp.f, h);
    accumulate<MU, R>(acc, uh, sg);
  }
}

// hops H..7: the loads of hop H + 1 are issued before hop H's arithmetic.  With TW
// (the t walk) hop 7's spinor (backward t) is tin, already in registers, and hop 6's
// (forward t) is handed back in tout for the next site of the walk.
template <int H, bool MF, bool L12, bool TW, bool ST>
__device__ __forceinline__ void mrhs_steps(Spinor<float>& acc, const Spinor<float>& p, const LinkPairT<MF>& lp,
                                           const HopCtx<float>& c, int row, int r, int nrhs, const Spinor<float>& tin,
                                           Spinor<float>& tout, const u4_t* st) {
  if constexpr (H < 7) {
    Spinor<float> pn;
    if constexpr (TW && H + 1 == 7)
      pn = tin;
    else
      pn = load_spinor<float>(c.in, mrhs_off(c.nb.j[H + 1], r, nrhs));
    LinkPairT<MF> ln = lp;
    if constexpr (((H + 1) & 1) == 0) {
      if constexpr (ST)
        load_pair_st<MF, L12>(st, (H + 1) >> 1, row, ln);
      else
        load_pair<MF, L12>(c, (H + 1) >> 1, row, ln);
    }
    mrhs_hop<H, MF, L12>(acc, p, lp, c);
    hop_fence<float>(acc);
    if constexpr (TW && H == 6) tout = p;
    mrhs_steps<H + 1, MF, L12, TW, ST>(acc, pn, ln, c, row, r, nrhs, tin, tout, st);
  } else {
    mrhs_hop<H, MF, L12>(acc, p, lp, c);
    hop_fence<float>(acc);
  }
}

// One output site per lane group: the eight hops, the clover epilogue of MODE and the
// store (lanes with ok == false store nothing).  TW: see mrhs_steps.
// ST: links and clover slots staged in LDS (st: this lane's site slot; rl: the lane's
// index within its site)
template <int MODE, bool MF, bool L12, bool TW, bool ST>
__device__ __forceinline__ void mrhs_site(const MrhsArgs& a, int i, int rc, bool ok, int row, const Spinor<float>& tin,
                                          Spinor<float>& tout, u4_t* st, int rl) {
  using R = float;
  const int vh = a.g.Vh;
  const int nrhs = a.nrhs;
  HopCtx<R> c;
  c.in = mrhs_field(a.in, nrhs, vh);
  c.links = a.links;
  c.lrows = L12 ? LINK12_ROWS : LINK_ROWS;
  c.vh = vh;
  c.loff = boff(i, c.lrows / CPE<R>);
  c.nb = neighbours(a.g, decode(a.g, i, a.p_out));
  c.sf = R(-1);  // D: forward (1 - g), backward (1 + g)
  c.sb = R(1);

  const Field cl = bfield(a.clov, CLOVER_ROWS / CPE<R>, vh);
  const uint32_t coff = boff(i, CLOVER_ROWS / CPE<R>);
  Spinor<R> acc;
  zero(acc);
  {
    const Spinor<R> p0 = load_spinor<R>(c.in, mrhs_off(c.nb.j[0], rc, nrhs));
    LinkPairT<MF> lp;
    if constexpr (ST) {
      stage_site<L12>(c, cl, coff, rl, a.lps, st);
      load_pair_st<MF, L12>(st, 0, row, lp);
    } else {
      load_pair<MF, L12>(c, 0, row, lp);
    }
    mrhs_steps<0, MF, L12, TW, ST>(acc, p0, lp, c, row, rc, nrhs, tin, tout, st);
  }
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) acc.c[sp][cc] = R(0.5) * acc.c[sp][cc];

  const uint32_t off = mrhs_off(i, rc, nrhs);
  auto cmul = [&](const Spinor<R>& v) {
    if constexpr (ST)
      return clover_mul_st(st, v);
    else
      return clover_mul<R>(cl, coff, v);
  };
  Spinor<R> res;
  if constexpr (MODE == M_HOP_CLINV) {
    res = cmul(acc);
  } else if constexpr (MODE == M_APPLY) {
    res = cmul(load_spinor<R, DDQ_OWN_AUX>(mrhs_field(a.x, nrhs, vh), off));
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) res.c[sp][cc] = res.c[sp][cc] - acc.c[sp][cc];
  } else {  // M_RICH
    Spinor<R> xx = load_spinor<R, DDQ_OWN_AUX>(mrhs_field(a.x, nrhs, vh), off);
    const Spinor<R> bb = load_spinor<R, DDQ_OWN_AUX>(mrhs_field(a.b, nrhs, vh), off);
    const Spinor<R> cx = cmul(xx);
#pragma unroll
    for (int sp = 0; sp < 4; ++sp)
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) {
        const cpx<R> rr = bb.c[sp][cc] - cx.c[sp][cc] + acc.c[sp][cc];
        xx.c[sp][cc] = xx.c[sp][cc] + a.omega * rr;
      }
    res = xx;
  }
  if (ok) store_spinor<R>(mrhs_field(a.out, nrhs, vh), off, res);  // out may alias x (in-place sweep)
}

// lane -> (site slot, right-hand side) of a wavefront whose sites start at `first` and
// end before `end`; lanes without a (site, right-hand side) of their own take a valid
// one for their loads (ok = false: no store)
struct LaneSite {
  int i, rc, row, rl, sl;
  bool ok;
};
__device__ __forceinline__ LaneSite lane_site(const MrhsArgs& a, int rg, int first, int end) {
  const int lane = (int)threadIdx.x & 63;
  const int sl = lane / a.lps, rl = lane - sl * a.lps;
  const int r = rg * a.rgs + rl;
  const bool site_ok = sl < a.spw && first + sl < end;
  LaneSite ls;
  ls.ok = site_ok && rl < a.rgs && r < a.nrhs;
  ls.i = site_ok ? first + sl : first;
  ls.rc = r < a.nrhs ? r : a.nrhs - 1;
  ls.row = lane & 3;  // the lane's link row in the matrix-core form
  ls.rl = rl;
  ls.sl = sl;
  return ls;
}

// LDS of the staged kernels: per wavefront stage_slots(lps) slots of ST_SITE_E elements
extern __shared__ u4_t mrhs_lds[];

template <int MODE, bool MF, bool L12, bool ST>
__global__ void __launch_bounds__(HOP_BLOCK)
__attribute__((amdgpu_waves_per_eu(MF ? DDQ_WAVES_MRHS_MFMA : DDQ_WAVES_MRHS_VALU)))
hop_mrhs_kernel(MrhsArgs a) {
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int blk = (int)blockIdx.x;
  const int gs = (HOP_BLOCK / 64) * a.spw;  // sites of a workgroup
  // sites of the launch: the whole lattice, or slices [t_lo, t_lo + t_cnt) when t_cnt > 0
  const int t_cnt = a.t_cnt > 0 ? a.t_cnt : a.g.L[3];
  int rg, base, end;
  if (a.order == MRHS_ORDER_SLAB) {
    const int local = blk >> 3, xcd = blk & 7;
    rg = local % a.ngroups;
    int q = local / a.ngroups;
    const int ng = (a.g.sT + gs - 1) / gs;
    const int n = (((xcd + 1) * ng) >> 3) - ((xcd * ng) >> 3);  // this XCD's groups per slice
    if (n <= 0 || q >= t_cnt * n) return;
    q += a.t_lo * n;
    if (!slab_group_n(a.g, xcd, q, gs, base, end)) return;
  } else {
    rg = blk % a.ngroups;
    base = a.t_lo * a.g.sT + (blk / a.ngroups) * gs;
    const int lim = (a.t_lo + t_cnt) * a.g.sT;
    if (base >= lim) return;
    end = min(base + gs, lim);
  }
  const int first = base + w * a.spw;
  if (first >= end) return;  // wavefront-uniform
  const LaneSite ls = lane_site(a, rg, first, end);
  u4_t* st = mrhs_lds + (size_t)(w * stage_slots(a.lps) + ls.sl) * ST_SITE_E;
  Spinor<float> unused;
  mrhs_site<MODE, MF, L12, false, ST>(a, ls.i, ls.rc, ls.ok, ls.row, unused, unused, st, ls.rl);
}

// The t walk.  A wavefront keeps the same spw sites of a t-slice (same x, y, z) and
// walks t in steps of two through `tsteps` slices of one parity of t, so the forward-t
// neighbour it loads for slice t is the backward-t neighbour of slice t + 2 and stays in
// registers.  Workgroups: XCD k (blk mod 8) owns piece k of every slice (the pieces of
// slab order); its workgroups take (segment of 2 tsteps slices, parity of t, group of
// gs sites of the piece, right-hand-side group), the group fastest, so the waves of an
// XCD walk t together over its piece and share each slice's spatial neighbours in L2.
template <int MODE, bool MF, bool L12, bool ST>
__global__ void __launch_bounds__(HOP_BLOCK)
__attribute__((amdgpu_waves_per_eu(MF ? DDQ_WAVES_MRHS_MFMA_TW : DDQ_WAVES_MRHS_VALU)))
hop_mrhs_tw_kernel(MrhsArgs a) {
  const int w = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 6);
  const int blk = (int)blockIdx.x;
  const int xcd = blk & 7;
  const int gs = (HOP_BLOCK / 64) * a.spw;
  const int P = a.g.sT;
  const int ng = (P + gs - 1) / gs;
  const int nmax = (ng + 7) >> 3;
  const int g0 = (xcd * ng) >> 3, n = (((xcd + 1) * ng) >> 3) - g0;
  int local = blk >> 3;
  const int rg = local % a.ngroups;
  local /= a.ngroups;
  const int gl = local % nmax;
  local /= nmax;
  const int tb = local & 1, seg = local >> 1;
  if (gl >= n) return;
  const int t0 = seg * 2 * a.tsteps + tb;
  if (t0 >= a.g.L[3]) return;
  const int off0 = (g0 + gl) * gs + w * a.spw;  // the wavefront's first site within a slice
  const int lim = min((g0 + gl) * gs + gs, P);
  if (off0 >= lim) return;  // wavefront-uniform
  Spinor<float> carry;
  for (int step = 0; step < a.tsteps; ++step) {
    const int t = t0 + 2 * step;
    if (t >= a.g.L[3]) break;
    const LaneSite ls = lane_site(a, rg, t * P + off0, t * P + lim);
    if (step == 0) {
      // backward-t neighbour of the first slice of the walk (wraps at t = 0)
      const int j = t == 0 ? ls.i + (a.g.L[3] - 1) * P : ls.i - P;
      carry = load_spinor<float>(mrhs_field(a.in, a.nrhs, a.g.Vh), mrhs_off(j, ls.rc, a.nrhs));
    }
    Spinor<float> next;
    u4_t* st = mrhs_lds + (size_t)(w * stage_slots(a.lps) + ls.sl) * ST_SITE_E;
    mrhs_site<MODE, MF, L12, true, ST>(a, ls.i, ls.rc, ls.ok, ls.row, carry, next, st, ls.rl);
    carry = next;
  }
}

// lanes per site and right-hand sides per group: groups of at most 16 right-hand
// sides, equal in size, each padded to a multiple of four lanes
bool mrhs_geometry(int nrhs, MrhsArgs& a) {
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS) return false;
  a.ngroups = (nrhs + 15) / 16;
  a.rgs = (nrhs + a.ngroups - 1) / a.ngroups;
  a.lps = (a.rgs + 3) / 4 * 4;
  a.spw = 64 / a.lps;
  return true;
}

long long mrhs_grid(const MrhsArgs& a) {
  const int gs = (HOP_BLOCK / 64) * a.spw;
  if (a.tsteps > 0) {
    const long long ng = (a.g.sT + gs - 1) / gs;
    const long long nseg = (a.g.L[3] / 2 + a.tsteps - 1) / a.tsteps;
    return 8LL * nseg * 2 * ((ng + 7) / 8) * a.ngroups;
  }
  const long long nt = a.t_cnt > 0 ? a.t_cnt : a.g.L[3];
  if (a.order == MRHS_ORDER_SLAB) {
    const long long ng = (a.g.sT + gs - 1) / gs;
    return 8LL * nt * ((ng + 7) / 8) * a.ngroups;
  }
  return (nt * a.g.sT + gs - 1) / gs * a.ngroups;
}

template <int MODE, bool MF, bool ST>
static hipError_t mrhs_launch_s(const MrhsArgs& a, dim3 grid, unsigned lds, hipStream_t s) {
  if (a.tsteps > 0) {
    if (a.link12)
      hipLaunchKernelGGL((hop_mrhs_tw_kernel<MODE, MF, true, ST>), grid, dim3(HOP_BLOCK), lds, s, a);
    else
      hipLaunchKernelGGL((hop_mrhs_tw_kernel<MODE, MF, false, ST>), grid, dim3(HOP_BLOCK), lds, s, a);
  } else if (a.link12) {
    hipLaunchKernelGGL((hop_mrhs_kernel<MODE, MF, true, ST>), grid, dim3(HOP_BLOCK), lds, s, a);
  } else {
    hipLaunchKernelGGL((hop_mrhs_kernel<MODE, MF, false, ST>), grid, dim3(HOP_BLOCK), lds, s, a);
  }
  return hipGetLastError();
}

template <int MODE, bool MF>
static hipError_t mrhs_launch_l(const MrhsArgs& a, hipStream_t s) {
  const long long nb = mrhs_grid(a);
  if (nb <= 0 || nb > 0x7fffffffLL) return hipErrorInvalidValue;
  // LDS: the staging slots, at least lds_kb (an occupancy cap)
  const unsigned st_bytes = a.stage ? (unsigned)((HOP_BLOCK / 64) * ((64 + a.lps - 1) / a.lps) * ST_SITE_E * 16) : 0u;
  const unsigned lds = std::max(st_bytes, (unsigned)a.lds_kb * 1024u);
  if (lds > 160u * 1024u) return hipErrorInvalidValue;
  return a.stage ? mrhs_launch_s<MODE, MF, true>(a, dim3((unsigned)nb), lds, s)
                 : mrhs_launch_s<MODE, MF, false>(a, dim3((unsigned)nb), lds, s);
}

template <int MODE>
static hipError_t mrhs_launch_e(const MrhsArgs& a, hipStream_t s) {
  return a.engine == MRHS_ENGINE_MFMA ? mrhs_launch_l<MODE, true>(a, s) : mrhs_launch_l<MODE, false>(a, s);
}

hipError_t launch_hop_mrhs(const MrhsArgs& a0, int mode, hipStream_t s) {
  MrhsArgs a = a0;
  if (!mrhs_geometry(a.nrhs, a)) return hipErrorInvalidValue;
  if (a.lds_kb < 0 || a.lds_kb > 160 || a.tsteps < 0 || a.tsteps > 4096) return hipErrorInvalidValue;
  if (a.t_lo < 0 || a.t_cnt < 0 || a.t_lo + a.t_cnt > a.g.L[3] || (a.t_cnt > 0 && a.tsteps > 0))
    return hipErrorInvalidValue;
  if ((uint64_t)a.g.Vh * 96u * (uint64_t)a.nrhs >= (1ULL << 32)) return hipErrorInvalidValue;
  switch (mode) {
    case M_HOP_CLINV: return mrhs_launch_e<M_HOP_CLINV>(a, s);
    case M_APPLY: return mrhs_launch_e<M_APPLY>(a, s);
    case M_RICH: return mrhs_launch_e<M_RICH>(a, s);
  }
  return hipErrorInvalidValue;
}

// ---------------------------------------------------------------------------
// layout changes: FP32 parity vectors [nrhs][6][V/2] 16-byte elements <-> the mrhs
// layout [V/2][6][nrhs]; pure data movement
// ---------------------------------------------------------------------------
__global__ void __launch_bounds__(256) k_mrhs_pack(const u4_t* __restrict__ src, u4_t* __restrict__ dst, int nrhs,
                                                   int vh, long long total) {
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const int r = (int)(e % nrhs);
    const long long ik = e / nrhs;
    const int k = (int)(ik % 6);
    const long long i = ik / 6;
    dst[e] = src[((long long)r * 6 + k) * vh + i];
  }
}
__global__ void __launch_bounds__(256) k_mrhs_unpack(const u4_t* __restrict__ src, u4_t* __restrict__ dst, int nrhs,
                                                     int vh, long long total) {
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < total; e += (long long)gridDim.x * 256) {
    const long long i = e % vh;
    const long long rk = e / vh;
    const int k = (int)(rk % 6);
    const int r = (int)(rk / 6);
    dst[e] = src[(i * 6 + k) * nrhs + r];
  }
}

hipError_t launch_mrhs_layout(const void* src, void* dst, int nrhs, int vh, bool to_mrhs, hipStream_t s) {
  const long long total = (long long)vh * 6 * nrhs;
  if (total <= 0) return hipSuccess;
  const long long want = (total + 255) / 256;
  const unsigned grid = (unsigned)(want < 65536 ? want : 65536);
  if (to_mrhs)
    hipLaunchKernelGGL(k_mrhs_pack, dim3(grid), dim3(256), 0, s, (const u4_t*)src, (u4_t*)dst, nrhs, vh, total);
  else
    hipLaunchKernelGGL(k_mrhs_unpack, dim3(grid), dim3(256), 0, s, (const u4_t*)src, (u4_t*)dst, nrhs, vh, total);
  return hipGetLastError();
}

}  // namespace ddq
