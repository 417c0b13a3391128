// sap.hip -- the block solves of SAP(n, m) (Sect. 2.4.1, Alg. 1), FP64.
//
// The lattice is cut into 4^4 blocks aligned at the origin; a block's colour is the
// parity of the sum of its block coordinates.  One workgroup solves one block of the
// launch's colour: D_kk e = r_k, D restricted to the block's sites (hops that leave the
// block dropped; a block that spans a whole direction keeps the wrap-around hops, with
// the antiperiodic sign in t), by odd-even preconditioning on the block (eq. 2 with the
// block's hopping terms) and m Minimal Residual steps on the block's Schur complement
// from zero; then x += e on the block's sites.  Thread j of the 128 owns the j-th even
// and the j-th odd site of the block (the checkerboard half index of the block's
// lexicographic site order); the hopping terms read the other parity's half-block
// vector from LDS, the links and clover blocks from HBM.
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
__device__ __forceinline__ void sap_hops(const Geo& g, const int lc[4], const cpx<double> (*v)[SAP_HALF],
                                         const HopCtx<double>& c, Spinor<double>& acc) {
  zero(acc);
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
    Spinor<double> p;
    if (inside) {
      const int jn = (nc[0] + SAP_B * (nc[1] + SAP_B * (nc[2] + SAP_B * nc[3]))) >> 1;
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int a = 0; a < 3; ++a) p.c[s][a] = v[3 * s + a][jn];
    } else {
      zero(p);
    }
    const Link<double> u = load_link_half<double>(link_field(c, mu), H & 1, c.loff);
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
    hop_fence<double>(acc);  // one hop at a time: bounds the live registers
  }
}

__device__ __forceinline__ void sap_put(cpx<double> (*v)[SAP_HALF], int j, const Spinor<double>& s) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) v[3 * sp + a][j] = s.c[sp][a];
}

__device__ __forceinline__ Spinor<double> sap_load_full(const d2_t* f, long long site) {
  Spinor<double> s;
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      const d2_t q = f[site * 12 + 3 * sp + a];
      s.c[sp][a] = {q.x, q.y};
    }
  return s;
}

__device__ __forceinline__ void sap_add_full(d2_t* f, long long site, const Spinor<double>& s) {
#pragma unroll
  for (int sp = 0; sp < 4; ++sp)
#pragma unroll
    for (int a = 0; a < 3; ++a) {
      d2_t q = f[site * 12 + 3 * sp + a];
      q.x += s.c[sp][a].r;
      q.y += s.c[sp][a].i;
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
  const pair<double>* links[2];  // FP64 links per parity
  const pair<double>* clov_e;    // A_ee (even sites)
  const pair<double>* clov_oi;   // A_oo^-1 (odd sites)
  int nb[4];                     // blocks per direction
  int colour;
  int m;  // Minimal Residual steps
};

__global__ void __launch_bounds__(SAP_HALF) k_sap_block(SapArgs a) {
  __shared__ cpx<double> ve[12][SAP_HALF];  // even half-block vector
  __shared__ cpx<double> vo[12][SAP_HALF];  // odd half-block vector
  __shared__ cpx<double> vx[12][SAP_HALF];  // the even half of the block correction (own slot only)
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
  const int ie = (int)(site_e >> 1), io = (int)(site_o >> 1);  // checkerboard indices
  const int vh = g.Vh;
  // hopping context of each of the thread's two sites: links, signs of the t hops
  HopCtx<double> ce, co;
  ce.links = a.links[0];
  co.links = a.links[1];
  ce.lrows = co.lrows = LINK_ROWS;
  ce.vh = co.vh = vh;
  ce.loff = boff(ie, LINK_ROWS);
  co.loff = boff(io, LINK_ROWS);
  ce.sf = co.sf = -1.0;  // D: forward (1 - g), backward (1 + g)
  ce.sb = co.sb = 1.0;
  const bool wrap_t = g.L[3] == SAP_B && g.antiperiodic;
  ce.nb.sgn_tf = (wrap_t && le[3] == SAP_B - 1) ? -1.f : 1.f;
  ce.nb.sgn_tb = (wrap_t && le[3] == 0) ? -1.f : 1.f;
  co.nb.sgn_tf = (wrap_t && lo[3] == SAP_B - 1) ? -1.f : 1.f;
  co.nb.sgn_tb = (wrap_t && lo[3] == 0) ? -1.f : 1.f;
  const Field Ce = bfield(a.clov_e, CLOVER_ROWS, vh);
  const Field Co = bfield(a.clov_oi, CLOVER_ROWS, vh);
  const uint32_t cofe = boff(ie, CLOVER_ROWS), cofo = boff(io, CLOVER_ROWS);

  Spinor<double> acc, rr, q;
  // eq. 2 on the block: b~_e = r_e - D_eo A_oo^-1 r_o = r_e + H_eo (A_oo^-1 r_o)
  sap_put(vo, j, clover_mul<double>(Co, cofo, sap_load_full(a.r, site_o)));
  __syncthreads();
  sap_hops(g, le, vo, ce, acc);
  rr = sap_load_full(a.r, site_e);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      rr.c[s][c] = rr.c[s][c] + 0.5 * acc.c[s][c];
      vx[3 * s + c][j] = {0.0, 0.0};
    }
  // Minimal Residual on the block Schur complement S = A_ee - H_eo A_oo^-1 H_oe
  for (int it = 0; it < a.m; ++it) {
    __syncthreads();  // every thread is done with ve and vo of the previous step
    sap_put(ve, j, rr);
    __syncthreads();
    sap_hops(g, lo, ve, co, acc);  // H_oe r
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) acc.c[s][c] = 0.5 * acc.c[s][c];
    sap_put(vo, j, clover_mul<double>(Co, cofo, acc));  // A_oo^-1 H_oe r
    __syncthreads();
    sap_hops(g, le, vo, ce, acc);  // H_eo A_oo^-1 H_oe r
    q = clover_mul<double>(Ce, cofe, rr);
    double d[3] = {0.0, 0.0, 0.0};  // q^H r, |q|^2
#pragma unroll
    for (int s = 0; s < 4; ++s)
#pragma unroll
      for (int c = 0; c < 3; ++c) {
        q.c[s][c] = q.c[s][c] - 0.5 * acc.c[s][c];
        const cpx<double> qv = q.c[s][c], rv = rr.c[s][c];
        d[0] += qv.r * rv.r + qv.i * rv.i;
        d[1] += qv.r * rv.i - qv.i * rv.r;
        d[2] += qv.r * qv.r + qv.i * qv.i;
      }
    sap_sum3(d, red);
    if (d[2] == 0.0) break;  // uniform: every thread holds the same sums
    const cpx<double> alpha = {d[0] / d[2], d[1] / d[2]};
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
      ve[3 * s + c][j] = q.c[s][c];
    }
  sap_add_full(a.x, site_e, q);
  __syncthreads();
  sap_hops(g, lo, ve, co, acc);
  rr = sap_load_full(a.r, site_o);
#pragma unroll
  for (int s = 0; s < 4; ++s)
#pragma unroll
    for (int c = 0; c < 3; ++c) acc.c[s][c] = rr.c[s][c] + 0.5 * acc.c[s][c];
  sap_add_full(a.x, site_o, clover_mul<double>(Co, cofo, acc));
}

hipError_t launch_sap_blocks(const Geo& g, const d2_t* r, d2_t* x, const void* links_e, const void* links_o,
                             const void* clov_e, const void* clov_oi, int colour, int m, hipStream_t s) {
  SapArgs a;
  a.g = g;
  a.r = r;
  a.x = x;
  a.links[0] = (const pair<double>*)links_e;
  a.links[1] = (const pair<double>*)links_o;
  a.clov_e = (const pair<double>*)clov_e;
  a.clov_oi = (const pair<double>*)clov_oi;
  long long nblk = 1;
  for (int mu = 0; mu < 4; ++mu) {
    if (g.L[mu] % SAP_B != 0) return hipErrorInvalidValue;
    a.nb[mu] = g.L[mu] / SAP_B;
    nblk *= a.nb[mu];
  }
  if (nblk > 0x7fffffffLL || m < 0) return hipErrorInvalidValue;
  a.colour = colour & 1;
  a.m = m;
  hipLaunchKernelGGL(k_sap_block, dim3((unsigned)nblk), dim3(SAP_HALF), 0, s, a);
  return hipGetLastError();
}

}  // namespace ddq
