// sap.hip -- the block solves of SAP(n, m) (Sect. 2.4.1, Alg. 1).
//
// The lattice is cut into 4^4 blocks aligned at the origin; a block's colour is the
// parity of the sum of its block coordinates.  One workgroup solves one block of the
// launch's colour: D_kk e = r_k, D restricted to the block's sites (hops that leave the
// block dropped; a block that spans a whole direction keeps the wrap-around hops, with
// the antiperiodic sign in t), by odd-even preconditioning on the block (eq. 2 with the
// block's hopping terms) and m Minimal Residual steps on the block's Schur complement
// from zero; then x += e on the block's sites.  The residual and the iterate are FP64
// full vectors; the block solve runs in R (FP64, or FP32 with FP32 links and clover),
// its dot products accumulated in FP64.  The links and clover blocks are read in SAP
// order: a copy of the link and clover fields with the 128 sites of one parity of each
// block at consecutive positions blockIdx * 128 + j (k_sap_reorder), so that every row
// a wavefront loads is one contiguous run.
//
// Two kernels:
// * k_sap_block_split (no block spans y, z or t; or FP32 with 12-real links): everything
//   the MR steps touch stays on chip -- the block's links in LDS, the clover blocks in
//   registers -- each site pair is split over two threads, and the colour's residual is
//   formed in the kernel's prologue (see the kernel).
// * k_sap_block (the other lattices: FP64, FP32 with 18-real links): 128 threads,
//   thread j owns the j-th even and the j-th odd site of the block (the checkerboard
//   half index of the block's lexicographic site order); the hopping terms read the
//   other parity's half-block vector from one LDS buffer, the links and clover blocks
//   from memory at every use.
#include "hop_common.h"

namespace ddq {

constexpr int SAP_B = 4;       // block extent per direction
constexpr int SAP_HALF = 128;  // sites of one parity in a block

// local coordinates of thread j's site of parity p (block origin at even coordinates,
// so local and global parities agree)
__device__ __forceinline__ void sap_local(int j, int p, int lc[4]) {
  lc[1] = (j >> 1) & 3;
  lc[2] = (j >> 3) & 3;
  lc[3] = (j >> 5) & 3;
  const int k = j & 1;
  lc[0] = 2 * k + ((p + lc[1] + lc[2] + lc[3]) & 1);
}

// sum of the block's hopping terms into a site at local coordinates lc: acc = sum over
// the 8 hops of (1 -/+ g_mu) U p(neighbour), p read from the other parity's half-block
// vector v[12][128] in LDS (zero for neighbours outside the block); `c` carries the
// site's links and the t-boundary signs
template <typename R>
__device__ __forceinline__ void sap_hops(const Geo& g, const int lc[4], const cpx<R> (*v)[SAP_HALF],
                                         const HopCtx<R>& c, Spinor<R>& acc) {
  zero(acc);
  Link<R> ub;
#pragma unroll
  for (int H = 0; H < 8; ++H) {
    const int mu = H >> 1;
    int nc[4] = {lc[0], lc[1], lc[2], lc[3]};
    nc[mu] += (H & 1) ? -1 : 1;
    bool inside = nc[mu] >= 0 && nc[mu] < SAP_B;
    if (!inside && g.L[mu] == SAP_B) {  // the block spans the direction: wrap inside it
      nc[mu] = (nc[mu] + SAP_B) % SAP_B;
      inside = true;
    }
    Spinor<R> p;
    if (inside) {
      const int jn = (nc[0] + SAP_B * (nc[1] + SAP_B * (nc[2] + SAP_B * nc[3]))) >> 1;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) p.c[s][a] = v[3 * s + a][jn];
    } else {
      zero(p);
    }
    Link<R> u;
    if constexpr (CPE<R> == 1) {
      u = load_link_half<R>(link_field(c, mu), H & 1, c.loff);
    } else if ((H & 1) == 0) {
      load_link_pair<R>(link_field(c, mu), c.loff, u, ub);
    } else {
      u = ub;
    }
    switch (H) {
      case 0: hop_compute<0, R>(acc, p, u, c); break;
      case 1: hop_compute<1, R>(acc, p, u, c); break;
      case 2: hop_compute<2, R>(acc, p, u, c); break;
      case 3: hop_compute<3, R>(acc, p, u, c); break;
      case 4: hop_compute<4, R>(acc, p, u, c); break;
      case 5: hop_compute<5, R>(acc, p, u, c); break;
      case 6: hop_compute<6, R>(acc, p, u, c); break;
      default: hop_compute<7, R>(acc, p, u, c); break;
    }
    hop_fence<R>(acc);  // one hop at a time: bounds the live registers
  }
}

template <typename R, int N>
__device__ __forceinline__ void sap_put(cpx<R> (*v)[N], int j, const Spinor<R>& s) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[3 * sp + a][j] = s.c[sp][a];
}

template <typename R>
__device__ __forceinline__ Spinor<R> sap_load_full(const d2_t* f, long long site) {
  Spinor<R> s;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const d2_t q = f[site * 12 + 3 * sp + a];
      s.c[sp][a] = {(R)q.x, (R)q.y};
    }
  return s;
}

template <typename R>
__device__ __forceinline__ void sap_add_full(d2_t* f, long long site, const Spinor<R>& s) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d2_t q = f[site * 12 + 3 * sp + a];
      q.x += (double)s.c[sp][a].r;
      q.y += (double)s.c[sp][a].i;
      f[site * 12 + 3 * sp + a] = q;
    }
  store_fence();
}

// sum over the workgroup's 128 threads of three doubles (two wavefronts)
__device__ __forceinline__ void sap_sum3(double v[3], double* red /* [2][3] */) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) red[3 * w + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = red[k] + red[3 + k];
}

struct SapArgs {
  Geo g;
  const d2_t* r;  // full residual b - D x (ABI full layout)
  d2_t* x;        // full iterate, updated on the blocks of `colour`
  SapResidualSrc res;  // the on-chip kernel's sources of r = b - D x when it forms r itself
  const void* links[2];  // links per parity, in the block solve's precision
  const void* clov_e;    // A_ee (even sites)
  const void* clov_oi;   // A_oo^-1 (odd sites)
  int nb[4];                     // blocks per direction
  int colour;
  int m;  // Minimal Residual steps
};

template <typename R>
__global__ void __launch_bounds__(SAP_HALF) k_sap_block(SapArgs a) {
  __shared__ cpx<R> vb[12][SAP_HALF];  // the other parity's half-block vector of the current hop
  __shared__ cpx<R> vx[12][SAP_HALF];  // the even half of the block correction (own slot only)
  __shared__ double red[6];
  const Geo& g = a.g;
  int bc[4];
  {
    int b = (int)blockIdx.x;
    bc[0] = b % a.nb[0];
    b /= a.nb[0];
    bc[1] = b % a.nb[1];
    b /= a.nb[1];
    bc[2] = b % a.nb[2];
    bc[3] = b / a.nb[2];
  }
  if (((bc[0] + bc[1] + bc[2] + bc[3]) & 1) != a.colour) return;  // uniform over the workgroup
  const int j = (int)threadIdx.x;
  int le[4], lo[4];
  sap_local(j, 0, le);
  sap_local(j, 1, lo);
  long long site_e, site_o;  // lexicographic site indices
  {
    int ge[4], go[4];
    for (int mu = 0; mu < 4; ++mu) {
      ge[mu] = SAP_B * bc[mu] + le[mu];
      go[mu] = SAP_B * bc[mu] + lo[mu];
    }
    site_e = ge[0] + (long long)g.L[0] * (ge[1] + (long long)g.L[1] * (ge[2] + (long long)g.L[2] * ge[3]));
    site_o = go[0] + (long long)g.L[0] * (go[1] + (long long)g.L[1] * (go[2] + (long long)g.L[2] * go[3]));
  }
  const int ss = (int)blockIdx.x * SAP_HALF + j;  // SAP-order position of both sites
  const int vh = g.Vh;
  constexpr int LR = LINK_ROWS;
  constexpr int CL_E = CLOVER_ROWS / CPE<R>;
  // hopping context of each of the thread's two sites: links, signs of the t hops
  HopCtx<R> ce, co;
  ce.links = (const pair<R>*)a.links[0];
  co.links = (const pair<R>*)a.links[1];
  ce.lrows = co.lrows = LR;
  ce.vh = co.vh = vh;
  ce.loff = boff(ss, LR / CPE<R>);
  co.loff = boff(ss, LR / CPE<R>);
  ce.sf = co.sf = R(-1);  // D: forward (1 - g), backward (1 + g)
  ce.sb = co.sb = R(1);
  const bool wrap_t = g.L[3] == SAP_B && g.antiperiodic;
  ce.nb.sgn_tf = (wrap_t && le[3] == SAP_B - 1) ? -1.f : 1.f;
  ce.nb.sgn_tb = (wrap_t && le[3] == 0) ? -1.f : 1.f;
  co.nb.sgn_tf = (wrap_t && lo[3] == SAP_B - 1) ? -1.f : 1.f;
  co.nb.sgn_tb = (wrap_t && lo[3] == 0) ? -1.f : 1.f;
  const Field Ce = bfield(a.clov_e, CL_E, vh);
  const Field Co = bfield(a.clov_oi, CL_E, vh);
  const uint32_t cofe = boff(ss, CL_E), cofo = boff(ss, CL_E);

  Spinor<R> acc, rr, q;
  // eq. 2 on the block: b~_e = r_e - D_eo A_oo^-1 r_o = r_e + H_eo (A_oo^-1 r_o)
  sap_put(vb, j, clover_mul<R>(Co, cofo, sap_load_full<R>(a.r, site_o)));
  __syncthreads();
  sap_hops<R>(g, le, vb, ce, acc);
  rr = sap_load_full<R>(a.r, site_e);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rr.c[s][c] = rr.c[s][c] + R(0.5) * acc.c[s][c];
      vx[3 * s + c][j] = {R(0), R(0)};
    }
  // Minimal Residual on the block Schur complement S = A_ee - H_eo A_oo^-1 H_oe
  for (int it = 0; it < a.m; ++it) {
    __syncthreads();  // every thread is done reading vb
    sap_put(vb, j, rr);
    __syncthreads();
    sap_hops<R>(g, lo, vb, co, acc);  // H_oe r
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.c[s][c] = R(0.5) * acc.c[s][c];
    const Spinor<R> t = clover_mul<R>(Co, cofo, acc);  // A_oo^-1 H_oe r
    __syncthreads();  // every thread is done reading r from vb
    sap_put(vb, j, t);
    __syncthreads();
    sap_hops<R>(g, le, vb, ce, acc);  // H_eo A_oo^-1 H_oe r
    q = clover_mul<R>(Ce, cofe, rr);
    double d[3] = {0.0, 0.0, 0.0};  // q^H r, |q|^2
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        q.c[s][c] = q.c[s][c] - R(0.5) * acc.c[s][c];
        const double qr = q.c[s][c].r, qi = q.c[s][c].i, rr_ = rr.c[s][c].r, ri = rr.c[s][c].i;
        d[0] += qr * rr_ + qi * ri;
        d[1] += qr * ri - qi * rr_;
        d[2] += qr * qr + qi * qi;
      }
    sap_sum3(d, red);
    if (d[2] == 0.0) break;  // uniform: every thread holds the same sums
    const cpx<R> alpha = {(R)(d[0] / d[2]), (R)(d[1] / d[2])};
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        vx[3 * s + c][j] = vx[3 * s + c][j] + alpha * rr.c[s][c];
        rr.c[s][c] = rr.c[s][c] - alpha * q.c[s][c];
      }
  }
  // eq. 2 on the block: e_o = A_oo^-1 (r_o - D_oe e_e) = A_oo^-1 (r_o + H_oe e_e)
  __syncthreads();
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      q.c[s][c] = vx[3 * s + c][j];
      vb[3 * s + c][j] = q.c[s][c];
    }
  sap_add_full(a.x, site_e, q);
  __syncthreads();
  sap_hops<R>(g, lo, vb, co, acc);
  rr = sap_load_full<R>(a.r, site_o);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.c[s][c] = rr.c[s][c] + R(0.5) * acc.c[s][c];
  sap_add_full(a.x, site_o, clover_mul<R>(Co, cofo, acc));
}

// ---------------------------------------------------------------------------
// The residual of Alg. 1 on the blocks of one colour: r = b - D x at every site of the
// colour's blocks (the sites the block solves read), FP64.  D x at a site is
// A x - 1/2 sum over the 8 hops of (1 -/+ g_mu) U x(neighbour) with the lattice's
// boundary conditions, the neighbours anywhere in the lattice.  Links and clover blocks
// (A_ee, A_oo: the undivided blocks) come from FP64 copies in SAP order, so each
// wavefront reads them as contiguous runs; x, b and r are the full vectors.  The
// on-chip block solves form it in their prologue; k_sap_residual writes it out for the
// other block-solve kernel.
// ---------------------------------------------------------------------------
// r at the site (parity q, half index j) of block blk at block coordinates bc
__device__ __forceinline__ Spinor<double> sap_residual_site(const Geo& g, const int bc[4], int blk, int q, int j,
                                                            const d2_t* b, const d2_t* x, const void* links,
                                                            const void* clov) {
  int lc[4], gc[4];
  sap_local(j, q, lc);
  for (int mu = 0; mu < 4; ++mu) gc[mu] = SAP_B * bc[mu] + lc[mu];
  auto lex = [&](const int c[4]) {
    return c[0] + (long long)g.L[0] * (c[1] + (long long)g.L[1] * (c[2] + (long long)g.L[2] * c[3]));
  };
  const long long site = lex(gc);
  const int ss = blk * SAP_HALF + j;
  HopCtx<double> c;
  c.links = (const pair<double>*)links;
  c.lrows = LINK_ROWS;
  c.vh = g.Vh;
  c.loff = boff(ss, LINK_ROWS);
  c.sf = -1.0;  // D: forward (1 - g), backward (1 + g)
  c.sb = 1.0;
  c.nb.sgn_tf = (g.antiperiodic && gc[3] == g.L[3] - 1) ? -1.f : 1.f;
  c.nb.sgn_tb = (g.antiperiodic && gc[3] == 0) ? -1.f : 1.f;
  long long nsite[8];
#pragma unroll
  for (int H = 0; H < 8; ++H) {
    const int mu = H >> 1;
    int nc[4] = {gc[0], gc[1], gc[2], gc[3]};
    nc[mu] += (H & 1) ? -1 : 1;
    if (nc[mu] < 0) nc[mu] += g.L[mu];
    if (nc[mu] >= g.L[mu]) nc[mu] -= g.L[mu];
    nsite[H] = lex(nc);
  }
  Spinor<double> acc;
  zero(acc);
#pragma unroll
  for (int H = 0; H < 8; ++H) {
    const Spinor<double> p = sap_load_full<double>(x, nsite[H]);
    const Link<double> u = load_link_half<double>(link_field(c, H >> 1), H & 1, c.loff);
    switch (H) {
      case 0: hop_compute<0, double>(acc, p, u, c); break;
      case 1: hop_compute<1, double>(acc, p, u, c); break;
      case 2: hop_compute<2, double>(acc, p, u, c); break;
      case 3: hop_compute<3, double>(acc, p, u, c); break;
      case 4: hop_compute<4, double>(acc, p, u, c); break;
      case 5: hop_compute<5, double>(acc, p, u, c); break;
      case 6: hop_compute<6, double>(acc, p, u, c); break;
      default: hop_compute<7, double>(acc, p, u, c); break;
    }
    hop_fence<double>(acc);
  }
  const Spinor<double> ax =
      clover_mul<double>(bfield(clov, CLOVER_ROWS, g.Vh), boff(ss, CLOVER_ROWS), sap_load_full<double>(x, site));
  const Spinor<double> bb = sap_load_full<double>(b, site);
  Spinor<double> r;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) r.c[sp][cc] = bb.c[sp][cc] - (ax.c[sp][cc] - 0.5 * acc.c[sp][cc]);
  return r;
}

// the block coordinates of workgroup k of a launch over one colour's blocks (bx fastest,
// (nb[0] + 1) / 2 a row); false for the spare workgroup of a row with an odd count
__device__ __forceinline__ bool sap_colour_block(const int nb[4], int colour, int k, int bc[4], int& blk) {
  const int hx = (nb[0] + 1) >> 1;
  int row = k / hx;
  bc[1] = row % nb[1];
  row /= nb[1];
  bc[2] = row % nb[2];
  bc[3] = row / nb[2];
  bc[0] = 2 * (k - (k / hx) * hx) + ((colour + bc[1] + bc[2] + bc[3]) & 1);
  blk = bc[0] + nb[0] * (bc[1] + nb[1] * (bc[2] + nb[2] * bc[3]));
  return bc[0] < nb[0];
}

struct SapResArgs {
  Geo g;
  d2_t* r;
  SapResidualSrc src;
  int nb[4];
  int colour;
};

// one workgroup of 256 threads per block (thread t: parity t / 128, half index t mod 128)
__global__ void __launch_bounds__(256) k_sap_residual(SapResArgs a) {
  int bc[4], blk;
  if (!sap_colour_block(a.nb, a.colour, (int)blockIdx.x, bc, blk)) return;  // uniform
  // the parity is uniform over a wavefront: its links and clover through scalar descriptors
  const int q = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 7), j = (int)threadIdx.x & (SAP_HALF - 1);
  const Spinor<double> r = sap_residual_site(a.g, bc, blk, q, j, a.src.b, a.src.x, a.src.links[q], a.src.clov[q]);
  int lc[4], gc[4];
  sap_local(j, q, lc);
  for (int mu = 0; mu < 4; ++mu) gc[mu] = SAP_B * bc[mu] + lc[mu];
  const long long site = gc[0] + (long long)a.g.L[0] * (gc[1] + (long long)a.g.L[1] * (gc[2] + (long long)a.g.L[2] * gc[3]));
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int cc = 0; cc < 3; ++cc) a.r[site * 12 + 3 * sp + cc] = d2_t{r.c[sp][cc].r, r.c[sp][cc].i};
}

// ---------------------------------------------------------------------------
// Block solves with the block's links in LDS across the MR steps: the forward hop of
// site x reads U_mu(x), the backward hop the neighbour's U_mu(x - mu) and applies its
// adjoint.  Two LDS forms of the links:
// * 12-real FP32 storage: rows 0 and 1 of all 1,024 forward links (48 KB), the third row
//   rebuilt at each hop; entry e of (direction mu, parity q, half index j) at
//   (e * 8 + 2 mu + q) * 128 + j;
// * 18-real storage (L18; FP32 or FP64; no block spans y, z or t): the whole matrices
//   of the 832 links a hop can use (59 KB in FP32, 120 KB in FP64) -- all of x, and of
//   y, z, t those whose site is not at the block's last coordinate in the direction
//   (that link leaves the block); entry e of (mu, q, compact index c) at
//   e * SAP_L18 + sap_l18_base(mu, q) + c.
// ---------------------------------------------------------------------------
constexpr int SAP_LK = 6;                        // entries of a link in the 12-real form
constexpr int SAP_L18 = 2 * (SAP_HALF + 3 * 96);  // links of the 18-real form

__device__ __forceinline__ int sap_lk_idx(int e, int mu, int q, int j) {
  return (e * 8 + 2 * mu + q) * SAP_HALF + j;
}
__device__ __forceinline__ int sap_l18_base(int mu, int q) {
  return mu == 0 ? q * SAP_HALF : 2 * SAP_HALF + (mu - 1) * 192 + q * 96;
}
// compact index of the link of direction mu at half index j (of a site whose coordinate
// in mu is at most 2, or mu = 0); clamped to a valid index for the others
__device__ __forceinline__ int sap_l18_c(int mu, int j) {
  if (mu == 0) return j;
  int c;
  if (mu == 1)
    c = (j & 1) + 2 * ((j >> 1) & 3) + 6 * (j >> 3);
  else if (mu == 2)
    c = (j & 7) + 8 * ((j >> 3) & 3) + 24 * (j >> 5);
  else
    c = j;
  return c < 95 ? c : 95;
}

// half index of hop H's neighbour of the site at local coordinates lc (wrapping inside
// a block that spans the direction); SAP_HALF, the index of the zero column of the LDS
// half-block vector, when the neighbour lies outside the block
__device__ __forceinline__ int sap_nbr(const Geo& g, const int lc[4], int H) {
  const int mu = H >> 1;
  int nc[4] = {lc[0], lc[1], lc[2], lc[3]};
  nc[mu] += (H & 1) ? -1 : 1;
  bool inside = (unsigned)nc[mu] < (unsigned)SAP_B;
  if (g.L[mu] == SAP_B) {  // uniform
    nc[mu] &= SAP_B - 1;
    inside = true;
  }
  return inside ? (nc[0] + SAP_B * (nc[1] + SAP_B * (nc[2] + SAP_B * nc[3]))) >> 1 : SAP_HALF;
}

// operands of hop H of the site (parity p, half index j): the neighbour's spinor from
// the half-block vector v (its zero column outside the block) and the link's stored
// entries; every lane reads, so the reads go out together
template <int H, bool L18, typename R>
__device__ __forceinline__ void sap_lds_loads(const Geo& g, const int lc[4], int p, int j,
                                              const cpx<R> (*v)[SAP_HALF + 1], const cpx<R>* lk,
                                              Spinor<R>& nb, Link<R>& u) {
  constexpr int MU = H >> 1;
  const int jn = sap_nbr(g, lc, H);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int a = 0; a < 3; ++a) nb.c[s][a] = v[3 * s + a][jn];
  // forward: the site's own link; backward: the neighbour's (outside the block, where
  // the spinor is zero, any link: the one at the site's own index)
  const int q = (H & 1) ? 1 - p : p, jl = ((H & 1) && jn < SAP_HALF) ? jn : j;
  if constexpr (L18) {
    const int o = sap_l18_base(MU, q) + sap_l18_c(MU, jl);
#pragma unroll
    for (int e = 0; e < 9; ++e) u.u[e] = lk[e * SAP_L18 + o];
  } else {
#pragma unroll
    for (int e = 0; e < SAP_LK; ++e) u.u[e] = lk[sap_lk_idx(e, MU, q, jl)];
  }
}

template <int H, bool L18, typename R>
__device__ __forceinline__ void sap_lds_hop(Spinor<R>& acc, const Spinor<R>& nb, Link<R> u,
                                            const HopCtx<R>& c) {
  if constexpr (!L18) su3_third_row(u);
  if constexpr (H & 1) {
    Link<R> d;
#pragma unroll
    for (int a = 0; a < 3; ++a)
#pragma unroll
      for (int b = 0; b < 3; ++b) d.u[3 * a + b] = conj(u.u[3 * b + a]);
    hop_compute<H, R>(acc, nb, d, c);
  } else {
    hop_compute<H, R>(acc, nb, u, c);
  }
}

// hops H..HE-1, the operands of hop H + 1 read before hop H's arithmetic
template <int H, int HE, bool L18, typename R>
__device__ __forceinline__ void sap_lds_steps(const Geo& g, const int lc[4], int p, int j,
                                              const cpx<R> (*v)[SAP_HALF + 1], const cpx<R>* lk,
                                              const HopCtx<R>& c, Spinor<R>& acc, const Spinor<R>& nb,
                                              const Link<R>& u) {
  if constexpr (H + 1 < HE) {
    Spinor<R> nn;
    Link<R> un;
    sap_lds_loads<H + 1, L18, R>(g, lc, p, j, v, lk, nn, un);
    sap_lds_hop<H, L18, R>(acc, nb, u, c);
    hop_fence<R>(acc);
    sap_lds_steps<H + 1, HE, L18, R>(g, lc, p, j, v, lk, c, acc, nn, un);
  } else {
    sap_lds_hop<H, L18, R>(acc, nb, u, c);
    hop_fence<R>(acc);
  }
}

// ---------------------------------------------------------------------------
// The kernel has two threads per site pair: 256 threads, thread (h, j) with
// h = threadIdx / 128 (uniform over a wavefront) and j = threadIdx mod 128.  Thread h
// sums the hops of directions 2h and 2h + 1 into a partial spinor; the partials meet in
// LDS, after which thread h owns spins 2h, 2h + 1 of its two sites: the rows clover
// block h acts on, the rows of the Minimal Residual vectors it updates.  In FP32 a
// workgroup takes 72 KB of LDS (12-real: links, the hop input, an exchange buffer;
// 18-real: links and the hop input, which then also carries the exchange), so two
// blocks share a compute unit with two wavefronts per SIMD; in FP64 145 KB, one block
// per compute unit.
// ---------------------------------------------------------------------------
constexpr int SAP_SPLIT = 2 * SAP_HALF;  // threads of a workgroup

// the hops of directions 2h, 2h + 1 (h uniform over the wavefront)
template <bool L18, typename R>
__device__ __forceinline__ void sap_hops_half(const Geo& g, const int lc[4], int p, int j, int h,
                                              const cpx<R> (*v)[SAP_HALF + 1], const cpx<R>* lk,
                                              const HopCtx<R>& c, Spinor<R>& acc) {
  zero(acc);
  Spinor<R> nb;
  Link<R> u;
  if (h == 0) {
    sap_lds_loads<0, L18, R>(g, lc, p, j, v, lk, nb, u);
    sap_lds_steps<0, 4, L18, R>(g, lc, p, j, v, lk, c, acc, nb, u);
  } else {
    sap_lds_loads<4, L18, R>(g, lc, p, j, v, lk, nb, u);
    sap_lds_steps<4, 8, L18, R>(g, lc, p, j, v, lk, c, acc, nb, u);
  }
}

// own[k] (k = 3 s + c: spin 2h + s, colour c) = the sum of both threads' partials;
// xb: exchange rows, row 6 h' + k written by the thread that does not own them (the
// caller orders the writes after every read of xb's previous contents)
template <int N, typename R>
__device__ __forceinline__ void sap_exchange(cpx<R> (*xb)[N], int h, int j, const Spinor<R>& acc,
                                             cpx<R> own[6]) {
  if (h == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) xb[6 + k][j] = acc.c[2 + k / 3][k % 3];
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) xb[k][j] = acc.c[k / 3][k % 3];
  }
  __syncthreads();
  if (h == 0) {
#pragma unroll
    for (int k = 0; k < 6; ++k) own[k] = acc.c[k / 3][k % 3] + xb[k][j];
  } else {
#pragma unroll
    for (int k = 0; k < 6; ++k) own[k] = acc.c[2 + k / 3][k % 3] + xb[6 + k][j];
  }
}

// rows 6 h .. 6 h + 5 of a site of a full FP64 vector
template <typename R>
__device__ __forceinline__ void sap_load_rows6(const d2_t* f, long long site, int h, cpx<R> o[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    const d2_t q = f[site * 12 + 6 * h + k];
    o[k] = {(R)q.x, (R)q.y};
  }
}
template <typename R>
__device__ __forceinline__ void sap_add_rows6(d2_t* f, long long site, int h, const cpx<R> s[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    d2_t q = f[site * 12 + 6 * h + k];
    q.x += (double)s[k].r;
    q.y += (double)s[k].i;
    f[site * 12 + 6 * h + k] = q;
  }
  store_fence();
}

template <typename R>
__device__ __forceinline__ void sap_put6(cpx<R> (*v)[SAP_HALF + 1], int h, int j, const cpx<R> s[6]) {
#pragma unroll
  for (int k = 0; k < 6; ++k) v[6 * h + k][j] = s[k];
}

// sum over the workgroup's 256 threads of three doubles (four wavefronts)
__device__ __forceinline__ void sap_sum3_4(double v[3], double* red /* [4][3] */) {
#pragma unroll
  for (int k = 0; k < 3; ++k)
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v[k] += __shfl_xor(v[k], off, 64);
  const int w = threadIdx.x >> 6;
  if ((threadIdx.x & 63) == 0)
#pragma unroll
    for (int k = 0; k < 3; ++k) red[3 * w + k] = v[k];
  __syncthreads();
#pragma unroll
  for (int k = 0; k < 3; ++k) v[k] = (red[k] + red[3 + k]) + (red[6 + k] + red[9 + k]);
}

// RES: the kernel forms r = b - D x at the block's sites itself (a.res), in a prologue
// whose memory traffic overlaps the other resident block's arithmetic; else it reads a.r
template <typename R, bool L18, bool RES>
__global__ void __launch_bounds__(SAP_SPLIT) __attribute__((amdgpu_waves_per_eu(sizeof(R) == 4 ? 2 : 1)))
k_sap_block_split(SapArgs a) {
  __shared__ cpx<R> lk[L18 ? 9 * SAP_L18 : SAP_LK * 8 * SAP_HALF];  // the block's links
  __shared__ cpx<R> vb[12][SAP_HALF + 1];  // hop input; column SAP_HALF zero
  __shared__ cpx<R> xb[L18 ? 1 : 12][SAP_HALF];  // partial sums in exchange (12-real form)
  __shared__ double red[12];
  const Geo& g = a.g;
  int bc[4], blk;
  if (!sap_colour_block(a.nb, a.colour, (int)blockIdx.x, bc, blk)) return;  // uniform
  const int j = (int)threadIdx.x & (SAP_HALF - 1);
  const int h = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 7);
  int le[4], lo[4];
  sap_local(j, 0, le);
  sap_local(j, 1, lo);
  long long site_e, site_o;
  {
    int ge[4], go[4];
    for (int mu = 0; mu < 4; ++mu) {
      ge[mu] = SAP_B * bc[mu] + le[mu];
      go[mu] = SAP_B * bc[mu] + lo[mu];
    }
    site_e = ge[0] + (long long)g.L[0] * (ge[1] + (long long)g.L[1] * (ge[2] + (long long)g.L[2] * ge[3]));
    site_o = go[0] + (long long)g.L[0] * (go[1] + (long long)g.L[1] * (go[2] + (long long)g.L[2] * go[3]));
  }
  cpx<R> ro[6], re[6];  // the thread's rows of the residual (r_o kept for the reconstruction)
  if constexpr (RES) {
    // r at the block's 256 sites (thread t: parity t / 128, half index j), passed to the
    // threads that own its rows through the LDS that the links take afterwards
    cpx<R>* rs = lk;  // [parity][12 rows][128 sites]
    {
      const int q = __builtin_amdgcn_readfirstlane((int)threadIdx.x >> 7);  // uniform over a wavefront
      const Spinor<double> rv =
          sap_residual_site(g, bc, blk, q, j, a.res.b, a.res.x, a.res.links[q], a.res.clov[q]);
#pragma unroll
      for (int sp = 0; sp < 4; ++sp)
#pragma unroll
        for (int cc = 0; cc < 3; ++cc)
          rs[(q * 12 + 3 * sp + cc) * SAP_HALF + j] = {(R)rv.c[sp][cc].r, (R)rv.c[sp][cc].i};
    }
    __syncthreads();
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      re[k] = rs[(6 * h + k) * SAP_HALF + j];
      ro[k] = rs[(12 + 6 * h + k) * SAP_HALF + j];
    }
    __syncthreads();  // the links overwrite rs
  } else {
    sap_load_rows6(a.r, site_o, h, ro);
    sap_load_rows6(a.r, site_e, h, re);
  }
  const int ss = blk * SAP_HALF + j;
  const int vh = g.Vh;
  constexpr int CL_E = CLOVER_ROWS / CPE<R>;
  const uint32_t loff = boff(ss, (L18 ? LINK_ROWS : LINK12_ROWS) / CPE<R>), coff = boff(ss, CL_E);
  // the forward links of directions 2h, 2h + 1 of both parities into LDS
  constexpr int LR = L18 ? LINK_ROWS : LINK12_ROWS;  // complex rows of a direction's field
#pragma unroll
  for (int q = 0; q < 2; ++q)
#pragma unroll
    for (int d = 0; d < 2; ++d) {
      const int mu = 2 * h + d;
      const Field U = bfield((const pair<R>*)a.links[q] + (size_t)mu * LR * field_vh(vh), LR / CPE<R>, vh);
      if constexpr (L18) {
        int lq[4];
        sap_local(j, q, lq);
        if (mu == 0 || lq[mu] < SAP_B - 1) {  // the links a hop inside the block uses
          constexpr int NR = (9 + CPE<R> - 1) / CPE<R> * CPE<R>;  // whole elements
          cpx<R> c10[NR];  // rows 0..8: U_mu(x)
          load_rows<R, DDQ_STREAM_AUX>(U, 0, NR, loff, c10);
          const int o = sap_l18_base(mu, q) + sap_l18_c(mu, j);
#pragma unroll
          for (int e = 0; e < 9; ++e) lk[e * SAP_L18 + o] = c10[e];
        }
      } else {
        cpx<R> c6[SAP_LK];
        load_rows<R, DDQ_STREAM_AUX>(U, 0, SAP_LK, loff, c6);
#pragma unroll
        for (int e = 0; e < SAP_LK; ++e) lk[sap_lk_idx(e, mu, q, j)] = c6[e];
      }
    }
  if (threadIdx.x < 12) vb[threadIdx.x][SAP_HALF] = {R(0), R(0)};
  cpx<R> cle[18], clo[18];  // clover block h of A_ee (even site) and of A_oo^-1 (odd site)
  load_rows<R, DDQ_STREAM_AUX>(bfield(a.clov_e, CL_E, vh), 18 * h, 18, coff, cle);
  load_rows<R, DDQ_STREAM_AUX>(bfield(a.clov_oi, CL_E, vh), 18 * h, 18, coff, clo);
  HopCtx<R> ce, co;
  ce.sf = co.sf = R(-1);
  ce.sb = co.sb = R(1);
  const bool wrap_t = g.L[3] == SAP_B && g.antiperiodic;
  ce.nb.sgn_tf = (wrap_t && le[3] == SAP_B - 1) ? -1.f : 1.f;
  ce.nb.sgn_tb = (wrap_t && le[3] == 0) ? -1.f : 1.f;
  co.nb.sgn_tf = (wrap_t && lo[3] == SAP_B - 1) ? -1.f : 1.f;
  co.nb.sgn_tb = (wrap_t && lo[3] == 0) ? -1.f : 1.f;

  Spinor<R> acc;
  cpx<R> rr[6], ex[6], t6[6], q6[6];
  // the partials of acc summed into the thread's rows; in the 18-real form through vb,
  // once every thread has read vb for its hops
  auto exchange = [&](cpx<R> own[6]) {
    if constexpr (L18) {
      __syncthreads();
      sap_exchange(vb, h, j, acc, own);
    } else {
      sap_exchange(xb, h, j, acc, own);
    }
  };
  // eq. 2 on the block: b~_e = r_e + H_eo (A_oo^-1 r_o)
  clover_block_apply<R>(clo, ro, t6);
  sap_put6(vb, h, j, t6);
  __syncthreads();  // the links and vb written
  sap_hops_half<L18, R>(g, le, 0, j, h, vb, lk, ce, acc);
  exchange(t6);
#pragma unroll
  for (int k = 0; k < 6; ++k) {
    rr[k] = re[k] + R(0.5) * t6[k];
    ex[k] = {R(0), R(0)};
  }
  // Minimal Residual on the block Schur complement S = A_ee - H_eo A_oo^-1 H_oe.  A
  // thread's stores into vb (its own rows of column j) need no barrier before them:
  // every other thread's reads of column j, in a hop, come before the barrier of the
  // exchange that follows that hop, and after the exchange only the thread itself reads
  // its own rows.
  for (int it = 0; it < a.m; ++it) {
    sap_put6(vb, h, j, rr);
    __syncthreads();
    sap_hops_half<L18, R>(g, lo, 1, j, h, vb, lk, co, acc);  // H_oe r
    exchange(q6);
#pragma unroll
    for (int k = 0; k < 6; ++k) q6[k] = R(0.5) * q6[k];
    clover_block_apply<R>(clo, q6, t6);  // A_oo^-1 H_oe r
    sap_put6(vb, h, j, t6);
    __syncthreads();
    sap_hops_half<L18, R>(g, le, 0, j, h, vb, lk, ce, acc);  // H_eo A_oo^-1 H_oe r
    exchange(t6);
    clover_block_apply<R>(cle, rr, q6);
    double d[3] = {0.0, 0.0, 0.0};  // q^H r, |q|^2
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      q6[k] = q6[k] - R(0.5) * t6[k];
      const double qr = q6[k].r, qi = q6[k].i, rr_ = rr[k].r, ri = rr[k].i;
      d[0] += qr * rr_ + qi * ri;
      d[1] += qr * ri - qi * rr_;
      d[2] += qr * qr + qi * qi;
    }
    sap_sum3_4(d, red);
    if (d[2] == 0.0) break;  // uniform: every thread holds the same sums
    const cpx<R> alpha = {(R)(d[0] / d[2]), (R)(d[1] / d[2])};
#pragma unroll
    for (int k = 0; k < 6; ++k) {
      ex[k] = ex[k] + alpha * rr[k];
      rr[k] = rr[k] - alpha * q6[k];
    }
  }
  // eq. 2 on the block: e_o = A_oo^-1 (r_o + H_oe e_e)
  sap_put6(vb, h, j, ex);
  sap_add_rows6(a.x, site_e, h, ex);
  __syncthreads();
  sap_hops_half<L18, R>(g, lo, 1, j, h, vb, lk, co, acc);
  exchange(t6);
#pragma unroll
  for (int k = 0; k < 6; ++k) t6[k] = ro[k] + R(0.5) * t6[k];
  clover_block_apply<R>(clo, t6, q6);
  sap_add_rows6(a.x, site_o, h, q6);
}

hipError_t launch_sap_residual(const Geo& g, const SapResidualSrc& src, d2_t* r, int colour, hipStream_t s) {
  SapResArgs a;
  a.g = g;
  a.r = r;
  a.src = src;
  long long rows = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (g.L[mu] % SAP_B != 0) return hipErrorInvalidValue;
    a.nb[mu] = g.L[mu] / SAP_B;
    if (mu > 0) rows *= a.nb[mu];
  }
  const long long nwg = rows * ((a.nb[0] + 1) / 2);
  if (nwg > 0x7fffffffLL) return hipErrorInvalidValue;
  a.colour = colour & 1;
  hipLaunchKernelGGL(k_sap_residual, dim3((unsigned)nwg), dim3(256), 0, s, a);
  return hipGetLastError();
}

// dst = src with its sites of parity p in SAP order: element row e of SAP position
// s = block * 128 + j comes from the site's checkerboard index (blocked fields of
// erows element rows)
__global__ void k_sap_reorder(Geo g, int p, int nb0, int nb1, int nb2, const u4_t* __restrict__ src,
                              u4_t* __restrict__ dst, int erows) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= (long long)g.Vh * erows) return;
  const int s = (int)(t % g.Vh), e = (int)(t / g.Vh);
  int b = s / SAP_HALF;
  const int j = s % SAP_HALF;
  int bc[4];
  bc[0] = b % nb0;
  b /= nb0;
  bc[1] = b % nb1;
  b /= nb1;
  bc[2] = b % nb2;
  bc[3] = b / nb2;
  int lc[4];
  sap_local(j, p, lc);
  long long lex = 0;
  for (int mu = 3; mu >= 0; --mu) lex = lex * g.L[mu] + (SAP_B * bc[mu] + lc[mu]);
  const int i = (int)(lex >> 1);
  dst[fidx(e, s, erows, g.Vh)] = src[fidx(e, i, erows, g.Vh)];
}

hipError_t launch_sap_reorder(const Geo& g, int parity, const void* src, void* dst, int erows, hipStream_t s) {
  for (int mu = 0; mu < 4; ++mu)
    if (g.L[mu] % SAP_B != 0) return hipErrorInvalidValue;
  const long long n = (long long)g.Vh * erows;
  const long long blocks = (n + 255) / 256;
  if (blocks > 0x7fffffffLL) return hipErrorInvalidValue;
  hipLaunchKernelGGL(k_sap_reorder, dim3((unsigned)blocks), dim3(256), 0, s, g, parity, g.L[0] / SAP_B,
                     g.L[1] / SAP_B, g.L[2] / SAP_B, (const u4_t*)src, (u4_t*)dst, erows);
  return hipGetLastError();
}

bool sap_on_chip(const Geo& g, int prec_f32, int link12) {
  return (prec_f32 && link12) || (g.L[1] > SAP_B && g.L[2] > SAP_B && g.L[3] > SAP_B);
}

template <typename R, bool L18>
static void launch_split(const SapArgs& a, bool res, dim3 grid, hipStream_t s) {
  if (res)
    hipLaunchKernelGGL((k_sap_block_split<R, L18, true>), grid, dim3(SAP_SPLIT), 0, s, a);
  else
    hipLaunchKernelGGL((k_sap_block_split<R, L18, false>), grid, dim3(SAP_SPLIT), 0, s, a);
}

hipError_t launch_sap_blocks(const Geo& g, int prec_f32, int link12, const d2_t* r, d2_t* x, const void* links_e,
                             const void* links_o, const void* clov_e, const void* clov_oi, int colour, int m,
                             const SapResidualSrc* res, hipStream_t s) {
  SapArgs a;
  a.g = g;
  a.r = r;
  a.x = x;
  if (res) {
    if (!sap_on_chip(g, prec_f32, link12)) return hipErrorInvalidValue;
    a.res = *res;
  } else {
    a.res = SapResidualSrc{};
  }
  a.links[0] = links_e;
  a.links[1] = links_o;
  a.clov_e = clov_e;
  a.clov_oi = clov_oi;
  long long nblk = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (g.L[mu] % SAP_B != 0) return hipErrorInvalidValue;
    a.nb[mu] = g.L[mu] / SAP_B;
    nblk *= a.nb[mu];
  }
  if (nblk > 0x7fffffffLL || m < 0) return hipErrorInvalidValue;
  a.colour = colour & 1;
  a.m = m;
  const dim3 grid((unsigned)nblk), block(SAP_HALF);
  // the on-chip kernel's grid: the blocks of one colour, (nb[0] + 1) / 2 of them a row in x
  const dim3 grid_c((unsigned)(nblk / a.nb[0] * ((a.nb[0] + 1) / 2)));
  const bool l18_fits = g.L[1] > SAP_B && g.L[2] > SAP_B && g.L[3] > SAP_B;  // no block spans y, z, t
  const bool rs = res != nullptr;
  if (!prec_f32 && l18_fits)
    launch_split<double, true>(a, rs, grid_c, s);
  else if (!prec_f32)
    hipLaunchKernelGGL(k_sap_block<double>, grid, block, 0, s, a);
  else if (link12)
    launch_split<float, false>(a, rs, grid_c, s);
  else if (l18_fits)
    launch_split<float, true>(a, rs, grid_c, s);
  else
    hipLaunchKernelGGL(k_sap_block<float>, grid, block, 0, s, a);
  return hipGetLastError();
}

}  // namespace ddq
