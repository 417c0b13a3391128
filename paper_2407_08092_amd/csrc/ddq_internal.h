// ddq_internal.h -- host-side declarations shared by the library's translation units.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "ddq_device.h"

namespace ddq {

// Epilogue of the hopping kernel.  The kernel computes h = H_{p, 1-p} in at every
// site of parity p (H restricted to rows of parity p, columns of parity 1-p) and
// then, with C the site's stored clover block (A_ee on even sites, A_oo^-1 on odd):
enum HopMode {
  M_HOP_CLINV = 0,  // out = C h                      u_o = A_oo^-1 H_oe x_e   (kernel A)
  M_RECON = 1,      // out = C (b + h)                x_o = A_oo^-1 (b_o + H_oe x_e)
  M_APPLY = 2,      // out = C x - h                  y_e = A_ee x_e - H_eo u_o (kernel B)
  M_RICH = 3,       // out = x + w (b - C x + h)      Richardson sweep, in place
  M_RESID = 4,      // out = b - C x + h              r = b - D_S x
  M_PREP = 5,       // out = b + h                    b~_e = b_e + H_eo u_o
  M_NMODES = 6
};

// Tile of the register-blocked multi-right-hand-side stencil (FP32): every thread
// handles nb right-hand sides of one site, so a link or clover entry is loaded
// once for nb spinors; g wavefronts of a workgroup take consecutive groups of
// right-hand sides of the same 64 sites (g = 1: 256 sites per workgroup); xmap = c > 0
// orders workgroups XCD by XCD: each XCD walks chunks of c consecutive site blocks,
// all right-hand-side groups of a block together, so a block's neighbour rows
// (+-z, +-t) are mostly read through the same L2 (xmap = 0: the dispatcher's
// round-robin order; xmap = XMAP_SLAB: slab order, slab_group).
// passes > 1 splits the right-hand sides into that many consecutive groups, one launch
// each (links and clover read once per pass, the neighbour rows of fewer right-hand
// sides in flight); lds_kb > 0 requests that much (unused) LDS per workgroup, which caps
// the workgroups resident on a compute unit and with them the sites in flight per XCD.
struct MrTile {
  int nb = 0;
  int g = 1;
  int xmap = 0;
  int passes = 1;
  int lds_kb = 0;
};

// workgroup blk -> (site block sb, right-hand-side group rg) of a launch with gr
// groups per site block; with chunk c > 0 the grid holds nsb padded to 8 c site blocks
__device__ __forceinline__ void tile_map(int blk, int gr, int c, int& sb, int& rg) {
  if (c <= 0) {
    sb = blk / gr;
    rg = blk % gr;
    return;
  }
  const int xcd = blk & 7, local = blk >> 3;
  const int per = c * gr;  // workgroups of one chunk
  const int chunk = local / per, within = local % per;
  sb = (chunk * 8 + xcd) * c + within / gr;
  rg = within % gr;
}
inline long long tile_grid(long long nsb, int gr, int c) {
  if (c > 0) nsb = (nsb + 8LL * c - 1) / (8LL * c) * (8LL * c);
  return nsb * gr;
}
constexpr int XMAP_SLAB = -1;
// site i of thread `lane` of workgroup blk and its right-hand-side group rg, for site
// blocks of spw sites (a multiple of 64; lane >> 6 is the thread's wavefront) and gr
// workgroups per site block; false if the thread has no site.  Slab order walks
// 64-site groups (slab_group) with all gr workgroups of a site block together.
__device__ __forceinline__ bool tile_site(const Geo& g, int blk, int gr, int c, int spw, int lane, int& i,
                                          int& rg) {
  if (c != XMAP_SLAB) {
    int sb;
    tile_map(blk, gr, c, sb, rg);
    i = sb * spw + lane;
    return i < g.Vh;
  }
  const int local = blk >> 3;
  rg = local % gr;
  const int q = (local / gr) * (spw >> 6) + __builtin_amdgcn_readfirstlane(lane >> 6);
  int base, end;
  if (!slab_group(g, blk & 7, q, base, end)) return false;
  i = base + (lane & 63);
  return i < end;
}
// workgroups of a tile_site launch
inline long long tile_grid_sites(const Geo& g, int spw, int gr, int c) {
  if (c == XMAP_SLAB) {
    const long long per = spw / 64;
    return 8LL * ((slab_groups_per_xcd(g) + per - 1) / per) * gr;
  }
  return tile_grid(((long long)g.Vh + spw - 1) / spw, gr, c);
}
constexpr int MR_MAX_NB = 4;

template <typename R>
struct HopArgs {
  Geo g;
  int p_out;                 // parity of the output sites
  const pair<R>* in;         // hopping input, parity 1 - p_out
  const pair<R>* links;      // 4 direction fields of LINK_ROWS complex rows, parity p_out
  const pair<R>* clov;       // clover field of CLOVER_ROWS complex rows, parity p_out
  const pair<R>* x;          // own-parity vector (APPLY, RICH, RESID)
  const pair<R>* b;          // own-parity right-hand side (RECON, RICH, RESID, PREP)
  pair<R>* out;
  R omega;
  int link12;                // FP32: links stored as their first two rows
  int nblk;                  // workgroups along x, padded to a multiple of 8 (one right-hand side)
  int nrhs;                  // right-hand sides of the launch
  long long rhs_stride;      // complex elements between right-hand sides
  MrTile tile;               // FP32 multi-right-hand-side tile (nb = 0: one right-hand side per thread)
  int t_lo, t_cnt;           // one right-hand side: only output sites of slices [t_lo, t_lo + t_cnt) (t_cnt 0: all)
};

#ifndef DDQ_HOP_BLOCK
#define DDQ_HOP_BLOCK 256
#endif
constexpr int HOP_BLOCK = DDQ_HOP_BLOCK;

template <typename R>
hipError_t launch_hop(const HopArgs<R>& a, int mode, bool dagger, int nrhs, hipStream_t s);
// the streaming ceiling of launch_hop's one-right-hand-side kernel for mode
// (M_HOP_CLINV, M_APPLY, M_RICH): the same bytes without gathers or arithmetic
template <typename R>
hipError_t launch_hop_stream(const HopArgs<R>& a, int mode, hipStream_t s);

// register-blocked FP32 multi-right-hand-side stencil for modes M_HOP_CLINV, M_APPLY
// and M_RICH (not daggered); a.tile.nb in [2, MR_MAX_NB] must divide nrhs.  Returns
// hipErrorInvalidValue for anything else (the caller falls back to launch_hop).
bool hop_rb_supported(int mode, bool dagger, int nrhs, const MrTile& t);
hipError_t launch_hop_rb(const HopArgs<float>& a, int mode, int nrhs, hipStream_t s);

// FP32 stencil on the mrhs layout (hop_mrhs.hip): right-hand sides interleaved per site,
// element (i, k, r) at (6 i + k) nrhs + r; modes M_HOP_CLINV, M_APPLY, M_RICH, not
// daggered.  The host fills everything up to lds_kb; launch_hop_mrhs derives the rest.
enum { MRHS_ENGINE_VALU = 0, MRHS_ENGINE_MFMA = 1 };
enum { MRHS_ORDER_PLAIN = 0, MRHS_ORDER_SLAB = 1, MRHS_ORDER_TWALK = 2 };
constexpr int MRHS_MAX_NRHS = 256;
struct MrhsArgs {
  Geo g;
  int p_out;
  const f2_t* in;
  const f2_t* links;
  const f2_t* clov;
  const f2_t* x;
  const f2_t* b;
  f2_t* out;
  float omega;
  int link12;
  int nrhs;
  int engine;   // MRHS_ENGINE_*: SU(3) products on the vector units or the matrix cores
  int order;    // MRHS_ORDER_*: workgroup order
  int lds_kb;   // LDS requested per workgroup (unused; caps resident workgroups)
  int tsteps;   // > 0: t walk, each wavefront takes that many slices of one parity of t
  int stage;    // 1: links and clover slots staged in LDS, shared by the lanes of a site
  int t_lo, t_cnt;  // slab and plain order: only output sites of slices [t_lo, t_lo + t_cnt) (t_cnt 0: all)
  // derived by mrhs_geometry
  int ngroups;  // right-hand-side groups (one workgroup each per site group)
  int rgs;      // right-hand sides per group (<= 16)
  int lps;      // lanes per site: rgs rounded up to a multiple of 4
  int spw;      // sites per wavefront: 64 / lps
};
bool mrhs_geometry(int nrhs, MrhsArgs& a);
hipError_t launch_hop_mrhs(const MrhsArgs& a, int mode, hipStream_t s);
// FP32 parity vectors [nrhs][6][V/2] <-> mrhs layout (to_mrhs selects the direction)
hipError_t launch_mrhs_layout(const void* src, void* dst, int nrhs, int vh, bool to_mrhs, hipStream_t s);

// 16-bit storage (FP16 or BF16 values, FP32 arithmetic): modes M_HOP_CLINV, M_APPLY,
// M_RICH, not daggered.  Parity vectors are [nrhs][3][V/2] 16-byte elements of four
// complex numbers; links 12-real; clover padded to 20 slots per block.
enum H16Kind { H16_F16 = 0, H16_BF16 = 1 };
struct Hop16Args {
  Geo g;
  int p_out;
  const u4_t* in;
  const u4_t* links;
  const u4_t* clov;
  const f2_t* clov32;  // non-null: read the FP32 clover blocks (CLOVER_ROWS rows) instead of clov
  const u4_t* x;
  const u4_t* b;
  u4_t* out;
  float omega;
  int nrhs;
  int nb;     // right-hand sides per thread, 1..3 (0: the largest of 3, 2, 1 dividing nrhs)
  int chunk;  // XCD order of the workgroups (tile_site): 0 dispatcher order, c > 0 chunks, XMAP_SLAB
};
hipError_t launch_hop16(int kind, const Hop16Args& a, int mode, hipStream_t s);
hipError_t launch_parity_to_h16(int kind, void* y, const d2_t* x, double scale, int nrhs, int vh, hipStream_t s);
hipError_t launch_parity_from_h16(int kind, d2_t* y, const void* x, double scale, int nrhs, int vh, hipStream_t s);
hipError_t launch_h16_to_f32(int kind, void* y, const void* x, float scale, int nrhs, int vh, hipStream_t s);
hipError_t launch_links_to_h16(int kind, const d2_t* in, void* out, int vh, hipStream_t s);
hipError_t launch_clover_to_h16(int kind, const d2_t* in, void* out, int vh, hipStream_t s);

// out = C v for every site of one parity (C = that parity's stored clover blocks)
template <typename R>
hipError_t launch_clover_only(const Geo& g, int nrhs, const pair<R>* clov, const pair<R>* v, pair<R>* out,
                              hipStream_t s);

// FP64 vector kernels (complex128 vectors of n elements)
hipError_t launch_dot_partial(const d2_t* V, long long vstride, int k, const d2_t* w, long long n,
                              d2_t* partial, int nbx, hipStream_t s);
hipError_t launch_reduce_partial(const d2_t* partial, int nbx, int k, d2_t* out, hipStream_t s);
hipError_t launch_update(d2_t* w, const d2_t* V, long long vstride, int k, const d2_t* h,
                         double sign, long long n, hipStream_t s);
hipError_t launch_norm2_partial(const d2_t* w, long long n, double* partial, int nbx, hipStream_t s);
hipError_t launch_reduce_real(const double* partial, int nbx, double* out, hipStream_t s);
hipError_t launch_scale(d2_t* out, const d2_t* in, double a, long long n, hipStream_t s);
hipError_t launch_scale_dev(d2_t* out, const d2_t* in, const double* inv_norm_dev, long long n,
                            hipStream_t s);
hipError_t launch_axpy(d2_t* y, double ar, double ai, const d2_t* x, long long n, hipStream_t s);
hipError_t launch_copy(d2_t* y, const d2_t* x, long long n, hipStream_t s);
hipError_t launch_scale_f32(f2_t* y, const f2_t* x, float a, long long n, hipStream_t s);

hipError_t launch_stream_copy(void* dst, const void* src, long long bytes, bool nontemporal, hipStream_t s);

// batched (nrhs systems, vector r at offset r * n; basis j at j * vstride)
hipError_t launch_dot_b(const d2_t* V, long long vstride, int k, const d2_t* w, long long n, int nrhs, d2_t* partial,
                        int nbx, d2_t* out, int ldo, hipStream_t s);
hipError_t launch_update_b(d2_t* w, const d2_t* V, long long vstride, int k, const d2_t* h, int ldh, double sign,
                           long long n, int nrhs, hipStream_t s);
hipError_t launch_norm2_b(const d2_t* w, long long n, int nrhs, double* partial, int nbx, double* out, hipStream_t s);
hipError_t launch_scale_b(d2_t* out, const d2_t* in, const double* f, long long n, int nrhs, hipStream_t s);
hipError_t launch_inv_norm_b(const double* hn, double* f, int nrhs, double tiny2, hipStream_t s);

// link force: insertions W (V x 54 complex) then per-link G (V x 4 x 9 complex) / F (V x 4 x 8)
hipError_t launch_force(const Geo& g, const d2_t* U, const d2_t* chi_e, const d2_t* lam_o, const d2_t* phi_e,
                        const d2_t* psi_o, double c_sw, d2_t* W, d2_t* G, double* F, int accumulate,
                        hipStream_t s);

// field kernels
hipError_t launch_pack_gauge_f64(const Geo& g, const d2_t* U, d2_t* out_even, d2_t* out_odd,
                                 hipStream_t s);
hipError_t launch_field_to_f32(const d2_t* in, void* out, int nfields, int crows, int vh, hipStream_t s);
hipError_t launch_links_to_f32_12(const d2_t* in, void* out, int vh, hipStream_t s);
hipError_t launch_parity_to_f32(void* y, const d2_t* x, int nrhs, int vh, hipStream_t s);
hipError_t launch_parity_to_f64(d2_t* y, const void* x, int nrhs, int vh, hipStream_t s);
// sources of the SAP residual r = b - D x (FP64 full vectors b, x; FP64 links per parity
// and undivided clover blocks A_ee, A_oo, in SAP order)
struct SapResidualSrc {
  const d2_t* b;
  const d2_t* x;
  const void* links[2];
  const void* clov[2];
};
// SAP block solves: for every 4^4 block of `colour`, m Minimal Residual steps on the
// block Schur complement of D_kk e = r_k, then x += e on the block (FP64 full vectors r,
// x); the block solve in FP64, or in FP32 (prec_f32) with FP32 links (12-real: link12)
// and clover, all in SAP order (launch_sap_reorder).  res: the block solves form r
// themselves from these sources (only where sap_on_chip holds); null: r is read
hipError_t launch_sap_blocks(const Geo& g, int prec_f32, int link12, const d2_t* r, d2_t* x, const void* links_e,
                             const void* links_o, const void* clov_e, const void* clov_oi, int colour, int m,
                             const SapResidualSrc* res, hipStream_t s);
// whether launch_sap_blocks solves this lattice's blocks on chip (and can form r itself)
bool sap_on_chip(const Geo& g, int prec_f32, int link12);
// r = b - D x (FP64 full vectors) at the sites of every 4^4 block of `colour`
hipError_t launch_sap_residual(const Geo& g, const SapResidualSrc& src, d2_t* r, int colour, hipStream_t s);
// copy of a blocked field of parity `parity` (erows element rows) into SAP order (the
// 128 sites of that parity of every 4^4 block consecutive), as launch_sap_blocks reads
// its links and clover
hipError_t launch_sap_reorder(const Geo& g, int parity, const void* src, void* dst, int erows, hipStream_t s);
// A_ee into clov_even, A_oo^-1 into clov_odd_inv and (when not null) A_oo into clov_odd
hipError_t launch_clover_build(const Geo& g, const d2_t* U, double c_sw, double m0,
                               d2_t* clov_even, d2_t* clov_odd_inv, d2_t* clov_odd, int* notpd, hipStream_t s);
hipError_t launch_clover_export(const Geo& g, const d2_t* packed, d2_t* dense, hipStream_t s);
template <typename R>
hipError_t launch_pack_parity(const Geo& g, int parity, int nrhs, const pair<R>* full, pair<R>* v,
                              hipStream_t s);
template <typename R>
hipError_t launch_unpack_parity(const Geo& g, int parity, int nrhs, const pair<R>* v, pair<R>* full,
                                hipStream_t s);

}  // namespace ddq
