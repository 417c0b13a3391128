/*
 * ddq.h -- C ABI of the odd-even Wilson-clover library for AMD Instinct MI355X (gfx950).
 *
 * The library applies and inverts the odd-even preconditioned Wilson-clover
 * Dirac operator of arXiv:2407.08092: the Schur complement
 *     D_S = D_ee - D_eo D_oo^-1 D_oe                                    (eq. 3)
 * of the even-first block form of D x = b                              (eq. 1),
 * its factorised inverse                                               (eq. 2),
 * the Richardson smoother of Alg. 4 and the restarted GMRES of Alg. 2 run on D_S.
 *
 * Operator (the paper names it in Sect. 2.3 but does not write it out; these are
 * the library's conventions):
 *   D psi(x) = A(x) psi(x) - H psi(x),
 *   H psi(x) = 1/2 sum_mu [(1 - g_mu) U_mu(x) psi(x+mu) + (1 + g_mu) U_mu(x-mu)^H psi(x-mu)],
 *   A(x)     = (4 + m0) + (i c_sw / 4) sum_{mu != nu} sigma_munu F_munu(x),
 *   F_munu   = (Q_munu - Q_munu^H) / 8, Q_munu = sum of the four plaquette leaves at x,
 * chiral gamma basis (g_k = [[0, -i s_k], [i s_k, 0]], g_4 = [[0, 1], [1, 0]],
 * g_5 = diag(1, 1, -1, -1)), so A(x) is two Hermitian 6x6 blocks (Sect. 2.4.5).
 * Periodic in x, y, z; antiperiodic in t when requested (a hop across the t
 * boundary carries -1).  A site is even when x+y+z+t is even (Sect. 2.4.5).
 *
 * Layouts (all complex numbers are (re, im) pairs of the stated real type):
 *   gauge links   U[t][z][y][x][mu][a][b]                      complex128
 *   full vector   psi[t][z][y][x][spin 4][colour 3]            complex128 or complex64
 *   parity vector rows sc = 3*spin + colour (12 rows) at site i = checkerboard
 *                 index of the site within its parity = (lexicographic index
 *                 x + Lx*(y + Ly*(z + Lz*t))) >> 1; right-hand-side stride
 *                 12*V/2 complex numbers.
 *                   DDQ_F64: complex128 v[rhs][sc][i] (row stride V/2).
 *                   DDQ_F32: complex64 v[rhs][sc/2][i][sc%2]: rows 2k and 2k+1 share
 *                   one 16-byte element per site, so every access is 16 bytes.
 *   clover export A[i][block 2][6][6] complex128, block 0 acting on spins 0,1 and
 *                 block 1 on spins 2,3, index 3*spin' + colour inside a block.
 *
 * Ownership: every field pointer is a device pointer owned by the caller, except
 * the gauge input of ddq_set_gauge, which may be a host pointer.  The library owns
 * its packed copies of links and clover blocks and its work buffers.  It allocates
 * device and pinned host memory only in ddq_create_lattice, ddq_set_gauge,
 * ddq_set_clover, ddq_reserve, ddq_tune_multi_rhs, ddq_autotune (through the tuner
 * it does not call: it only reads and writes the cache) and, for a batch, in
 * ddq_batch_create and ddq_batch_reserve; ddq_destroy_lattice / ddq_batch_destroy
 * free it.  Every other call -- apply, smooth, prepare, reconstruct, the solvers,
 * the force -- allocates nothing: when its work space exceeds what was reserved it
 * returns DDQ_ERR_STATE and does nothing.  ddq_set_gauge / ddq_set_clover reserve
 * one right-hand side of apply and smooth in every stored precision.
 *
 * Streams: every call enqueues its work on the lattice's stream and returns
 * without waiting, except ddq_set_clover, ddq_get_clover, ddq_estimate_lambda_max
 * and ddq_oe_gmres_solve, which synchronise that stream.  One thread at a time
 * per lattice handle.
 *
 * Errors: every call returns a ddq_status; no exception crosses the ABI.  On an
 * error ddq_last_error() returns a message for the calling thread.
 */
#ifndef DDQ_H
#define DDQ_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct ddq_lattice ddq_lattice;

/* Arithmetic of a call.  DDQ_F64: complex128 vectors, FP64 links and clover.
 * DDQ_F32: complex64 vectors, FP32 links and clover (blocks inverted in FP64,
 * then rounded).  DDQ_F16 / DDQ_BF16: 16-bit storage of vectors, links (12-real)
 * and clover blocks (rounded from FP64) with FP32 arithmetic: the lower-precision
 * storage the paper leaves to future work (Sect. 4).  16-bit parity vectors are
 * [rhs][sc/4][i][sc%4] complex pairs of 16-bit values (four complex numbers per
 * 16-byte element); FP16's range (normal numbers 6.1e-5 .. 65504) is the
 * caller's to respect.  Narrowing from FP64 rounds to nearest even: FP16 in one
 * rounding, BF16 through FP32 (two roundings); widening is exact.  The 16-bit path applies D_S and runs the Richardson
 * smoother (not daggered) and serves as the GMRES preconditioner's storage. */
enum ddq_prec { DDQ_F64 = 0, DDQ_F32 = 1, DDQ_F16 = 2, DDQ_BF16 = 3 };

enum ddq_status {
  DDQ_OK = 0,
  DDQ_NOT_CONVERGED = 1,   /* solver stopped at max_cycles; x holds the last iterate */
  DDQ_ERR_ARG = -1,        /* bad argument (odd extent, null pointer, bad precision ...) */
  DDQ_ERR_STATE = -2,      /* call out of order (apply before set_gauge / set_clover) */
  DDQ_ERR_HIP = -3,        /* a HIP runtime call failed */
  DDQ_ERR_OOM = -4,        /* device allocation failed */
  DDQ_ERR_NOT_PD = -5,     /* a 6x6 clover block is not positive definite */
  DDQ_ERR_NONFINITE = -6   /* NaN or Inf met in a residual norm */
};

/* storage_flags of ddq_set_gauge: which link precisions to materialise.  FP64
 * links are always kept (the outer residual of the solver uses them).
 * DDQ_STORE_F32_LINK12 stores the FP32 links as their first two rows only and
 * rebuilds the third from SU(3) unitarity (row 2 = conj(row 0 x row 1)) inside
 * the kernels: one third fewer link bytes.  DDQ_STORE_F16 / DDQ_STORE_BF16 add
 * 16-bit 12-real links (and, at ddq_set_clover, 16-bit clover blocks). */
enum { DDQ_STORE_F64 = 1, DDQ_STORE_F32 = 2, DDQ_STORE_F32_LINK12 = 4, DDQ_STORE_F16 = 8, DDQ_STORE_BF16 = 16 };

/* Lattice of extents dims = {Lx, Ly, Lz, Lt}, each even and >= 2.  The kernels
 * address every field through 32-bit buffer descriptors; the largest field, the
 * FP64 clover blocks of one parity (576 bytes a site), must stay below 4 GiB, so
 * V/2 (rounded up to a multiple of 64) must not exceed 7,456,512 sites (48^3 x 96
 * has 5,308,416); larger lattices are refused with DDQ_ERR_ARG before anything is
 * allocated.  t_antiperiodic != 0 selects antiperiodic t.
 * hip_stream: a hipStream_t (NULL = the null stream). */
int ddq_create_lattice(const int dims[4], int t_antiperiodic, void* hip_stream,
                       ddq_lattice** out);
int ddq_destroy_lattice(ddq_lattice* lat);
int ddq_set_stream(ddq_lattice* lat, void* hip_stream);
/* volume V and half volume V/2 */
int ddq_lattice_size(const ddq_lattice* lat, int64_t* volume, int64_t* half_volume);

/* Work space of the calls that follow (they allocate nothing themselves).  The
 * reservation only grows: every call raises it to at least these limits and
 * allocates what the lattice's stored precisions then need; ddq_set_gauge applies it
 * to precisions stored later.
 *   max_nrhs  right-hand sides of ddq_apply_schur, ddq_richardson_smooth,
 *             ddq_backward_apply (u_o in every stored precision), ddq_oe_prepare /
 *             ddq_oe_reconstruct and, with DDQ_RESERVE_FULL, ddq_apply_dirac /
 *             ddq_oe_smoother (1 .. 4096)
 *   max_m     GMRES / FGMRES cycle length (0 .. 128)
 *   what      DDQ_RESERVE_SOLVE: ddq_oe_gmres_solve (2 max_m + 4 FP64 and 3 FP32
 *             parity vectors; several right-hand sides are solved one after the
 *             other in this space);  DDQ_RESERVE_FULL: the full operator, the
 *             odd-even smoother and ddq_fgmres_solve (8 FP64 and 2 FP32 parity
 *             vectors per right-hand side, 2 max_m + 2 full FP64 vectors);
 *             DDQ_RESERVE_SAP: ddq_sap_smooth / ddq_fgmres_sap_solve (SAP-ordered
 *             copies of links and clover, the residual work space, FGMRES);
 *             DDQ_RESERVE_FORCE: ddq_backward_link_force (V x 54 complex128
 *             insertions and two parity vectors)
 * Returns DDQ_ERR_OOM when the device memory does not suffice (the reservation then
 * keeps what it had). */
enum { DDQ_RESERVE_SOLVE = 1, DDQ_RESERVE_FULL = 2, DDQ_RESERVE_SAP = 4, DDQ_RESERVE_FORCE = 8 };
int ddq_reserve(ddq_lattice* lat, int max_nrhs, int max_m, unsigned what);

/* Gauge links U (canonical layout, SU(3), complex128; host pointer when
 * U_on_device == 0).  Packs them into the library's per-parity layout in the
 * precisions selected by storage_flags.  Invalidates the clover term. */
int ddq_set_gauge(ddq_lattice* lat, const void* U, int U_on_device, unsigned storage_flags);

/* Builds the clover blocks A(x) on the GPU in FP64 (Sect. 2.3 operator), keeps
 * A_ee and inverts every odd-site 6x6 block by Cholesky in FP64 (Sect. 2.4.5:
 * storing D_oo^-1 is cheap); then rounds to every stored link precision.
 * Returns DDQ_ERR_NOT_PD if a block is not positive definite. */
int ddq_set_clover(ddq_lattice* lat, double c_sw, double m0);

/* Exports A_ee and A_oo^-1 (FP64) in the clover export layout; device pointers,
 * each V/2 * 72 complex128. Either may be NULL. */
int ddq_get_clover(ddq_lattice* lat, void* A_ee, void* A_oo_inv);

/* Full vector <-> parity vector (parity 0 = even, 1 = odd), nrhs right-hand
 * sides, vectors complex128 (DDQ_F64) or complex64 (DDQ_F32). */
int ddq_pack_parity(ddq_lattice* lat, int prec, int nrhs, int parity,
                    const void* full, void* v);
int ddq_unpack_parity(ddq_lattice* lat, int prec, int nrhs, int parity,
                      const void* v, void* full);

/* Parity vectors between the FP64 and FP32 layouts (rounding to FP32 or exact
 * widening); equal precisions copy.  src and dst must not overlap. */
int ddq_convert_parity(ddq_lattice* lat, int nrhs, int src_prec, const void* src, int dst_prec, void* dst);

/* y_e = D_S x_e (eq. 3), or D_S^H x_e = g_5 D_S g_5 x_e when dagger != 0, for
 * nrhs parity vectors.  x_e and y_e must not overlap. */
int ddq_apply_schur(ddq_lattice* lat, int prec, int nrhs, const void* x_e, void* y_e,
                    int dagger);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): ddq_apply_schur with the same
 * arguments, result and kernels, whose work space for u_o comes from a fixed 64 MiB
 * device array built into the library (one copy per GPU, held until the process ends)
 * instead of the lattice's reservation.  It calls no hipMalloc, hipFree or other
 * allocating routine, and the per-kernel profiler does not record it.  Limit:
 * nrhs * V/2 * 12 * (16, 8 or 4 bytes for DDQ_F64, DDQ_F32 or 16-bit) <= 64 MiB, e.g.
 * one FP64 or two FP32 right-hand sides of 24^3 x 48; larger requests return
 * DDQ_ERR_ARG.  Call it on the device the lattice was created on (else
 * DDQ_ERR_STATE).  Every call on one GPU shares that array: calls that overlap in time
 * on one GPU (two streams, two threads, two lattices) race and must be ordered by the
 * caller; nothing in the array needs to start at zero (u_o is written in full before
 * it is read). */
int ddq_apply_schur_noalloc(ddq_lattice* lat, int prec, int nrhs, const void* x_e, void* y_e,
                            int dagger);

/* Alg. 4 on D_S: nsweeps times x_e <- x_e + omega (b_e - D_S x_e), in place
 * (x_e: in x^(0), out x^(n)).  omega is used as given; Alg. 4's
 * omega = delta / |lambda_max| is formed by the caller (see
 * ddq_estimate_lambda_max). */
int ddq_richardson_smooth(ddq_lattice* lat, int prec, int nrhs, void* x_e, const void* b_e,
                          int nsweeps, double omega);

/* One-right-hand-side Richardson sweeps and Schur applies (FP64 / FP32
 * ddq_richardson_smooth and ddq_apply_schur with nrhs = 1, daggered too) on nc ranges of
 * t-slices (1 <= nc <= Lt; 0, the default, chooses for FP32 lattices whose u_o exceeds 128
 * MiB nc ranges of about 40 MiB of u_o each (13 at 48^3 x 96), else one): each launches
 * kernel A and kernel B per range, ordered so that the result is that of eq. 3 / Alg. 4
 * bit for bit (every B
 * reads u_o of the old x; every A reads x before its neighbour range is updated) while the
 * u_o rows of a range are read one launch after they were written, from the Infinity
 * Cache instead of HBM.  The interleaved multi-right-hand-side calls (ddq_mrhs_*) use the
 * ranges only when nc > 0 is set here, and never with their t walk. */
int ddq_set_sweep_chunks(ddq_lattice* lat, int nc);

/* Clover blocks of the 16-bit (DDQ_F16 / DDQ_BF16) stencil: fp32 = 0 reads the 16-bit
 * copies of A_ee and A_oo^-1 (rounded from FP64, 944 bytes per even site per Schur
 * apply in all), fp32 = 1 the FP32 blocks (links and spinors stay 16-bit: 1,200 bytes
 * per even site); needs DDQ_STORE_F32 (else DDQ_ERR_STATE), and a later ddq_set_gauge
 * without it returns to 0.  Half precision is the lower precision the paper names as
 * future work (Sect. 4). */
int ddq_set_h16_clover(ddq_lattice* lat, int fp32);

/* Tiles of the FP32 multi-right-hand-side stencil (nrhs >= 2 in ddq_apply_schur
 * and ddq_richardson_smooth, not daggered).  The operator is that of Sect. 2.4.5
 * applied to nrhs vectors that share the links and clover blocks; the paper applies
 * one vector at a time and names several right-hand sides as a way to make the
 * block applications cache-friendly (Sect. 3.3); the tiling is this library's.
 *   nb       right-hand sides per thread (links and clover slots loaded once for
 *            nb spinors); 1..4 and dividing nrhs.  0: one right-hand side per
 *            thread, 64 sites x 4 right-hand sides per workgroup, the workgroups
 *            in the order xcd_map (the default, with slab order; also the FP64
 *            kernels' and the modes the tiles do not cover).
 *   waves    1: a workgroup covers 256 sites; 4: its four wavefronts take four
 *            consecutive right-hand-side groups of the same 64 sites
 *   xcd_map  c in 1..1024: workgroups are ordered XCD by XCD, each XCD walking
 *            chunks of c consecutive site blocks with every right-hand-side group
 *            of a block together, so neighbour rows are read through one L2;
 *            0: the dispatcher's round-robin order; -1: slab order (every
 *            t-slice cut into eight pieces of whole 64-site groups, XCD k walking
 *            piece k of each slice in t order, so z- and t-neighbours share its
 *            L2; the order of the one-right-hand-side kernels).  The 16-bit
 *            kernels use the xcd_map of the tile set for the same nrhs, slab
 *            order if none.
 *   passes   (nb >= 1) the right-hand sides are split into this many consecutive
 *            groups, one launch each: links and clover are read once per pass while
 *            the neighbour rows of fewer right-hand sides compete for the L2; must
 *            divide nrhs, with nb dividing nrhs / passes
 *   lds_kb   (nb >= 1) LDS requested per workgroup (0 .. 160 KB; the kernel uses none):
 *            caps the workgroups resident on a compute unit, and so the sites whose
 *            neighbour rows are in flight on an XCD at once
 *   ms       (tuner output) mean time of one Richardson sweep with this tile
 * ddq_set_multi_rhs_tile: use `tile` for launches with nrhs right-hand sides.
 * ddq_tune_multi_rhs: the autotuner.  Times one FP32 Richardson sweep (kernel A +
 *   kernel B) for every valid tile, `reps` times each (HIP events on the lattice's
 *   stream, zeroed work vectors), keeps the fastest for nrhs, and reports up to
 *   max_results timed candidates (n_results receives their count) and the choice.
 *   Allocates two FP32 work vectors of nrhs right-hand sides on first use;
 *   synchronises the stream.  A batch solve tunes every (lattice, nrhs) it meets
 *   untuned. */
typedef struct {
  int nb;
  int waves;
  int xcd_map;
  double ms;
  int passes;
  int lds_kb;
} ddq_mr_tile;

int ddq_set_multi_rhs_tile(ddq_lattice* lat, int nrhs, const ddq_mr_tile* tile);
int ddq_tune_multi_rhs(ddq_lattice* lat, int nrhs, int reps, ddq_mr_tile* results, int max_results,
                       int* n_results, ddq_mr_tile* chosen);

/* Several right-hand sides in the interleaved ("mrhs") layout, FP32 (DDQ_F32 links
 * and clover; 12-real when the lattice stores them so).  The operator is D_S of eq. 3
 * on nrhs vectors that share the links and clover blocks; the paper names several
 * right-hand sides as the way to make block applications cache-friendly (Sect. 3.3).
 * Layout of an mrhs parity vector (complex64, device): [V/2][6][nrhs][2], i.e. the
 * 16-byte element holding rows 2k, 2k+1 (row = 3 spin + colour) of right-hand side r
 * at checkerboard site i sits at element (6 i + k) nrhs + r: all right-hand sides of a
 * site are one contiguous run.  nrhs in 1..256, and V/2 x 96 x nrhs bytes below 4 GiB.
 *   engine  DDQ_ENGINE_VALU: the SU(3) products on the vector units;
 *           DDQ_ENGINE_MFMA: on the matrix cores (v_mfma_f32_4x4x1_16b_f32, one 4 x 4
 *           outer-product block per four right-hand sides of a site); both give the same
 *           operator to FP32 rounding.
 * ddq_mrhs_pack / ddq_mrhs_unpack: FP32 parity vectors [nrhs][6][V/2][2] (the layout of
 *   ddq_apply_schur) to and from the mrhs layout (data movement only; src and dst must not
 *   overlap).
 * ddq_mrhs_apply_schur: y = D_S x (x and y must not overlap).
 * ddq_mrhs_richardson_smooth: Alg. 4, nsweeps times x <- x + omega (b - D_S x), in place.
 *   Both need the work space of ddq_reserve with max_nrhs >= nrhs (u_o in FP32).
 * ddq_mrhs_set_launch: workgroup order (0: plain site order, 1: slab order, the default:
 *   every t-slice cut into eight pieces, XCD k walking piece k of each slice in t order;
 *   2: t walk: a wavefront keeps its sites' x, y, z and walks tsteps slices of one parity
 *   of t (t, t + 2, ...; 1 <= tsteps <= Lt / 2), carrying the forward-t neighbour it
 *   loaded as the next slice's backward-t neighbour, the XCDs owning the pieces of slab
 *   order) and LDS requested per workgroup (0..160 KB; the kernels use none: it caps the
 *   workgroups resident on a compute unit).  tsteps is ignored unless order = 2.
 *   stage = 1 (the default) stages each site's links and clover slots in LDS: the lanes of
 *   a site load every 16-byte element once between them and read it from LDS, instead of
 *   each lane loading all of them (stage = 0; the LDS of the slots, 864 bytes per site of
 *   a workgroup, counts towards lds_kb).  Defaults: order 1, lds_kb 0, stage 1. */
enum { DDQ_ENGINE_VALU = 0, DDQ_ENGINE_MFMA = 1 };
int ddq_mrhs_pack(ddq_lattice* lat, int nrhs, const void* src, void* dst);
int ddq_mrhs_unpack(ddq_lattice* lat, int nrhs, const void* src, void* dst);
int ddq_mrhs_apply_schur(ddq_lattice* lat, int nrhs, const void* x_e, void* y_e, int engine);
int ddq_mrhs_richardson_smooth(ddq_lattice* lat, int nrhs, void* x_e, const void* b_e, int nsweeps, double omega,
                               int engine);
int ddq_mrhs_set_launch(ddq_lattice* lat, int order, int lds_kb, int tsteps, int stage);

/* Persisted tiles.  cache_json_path names a JSON file {"ddq_autotune": 1, "tiles":
 * [{"key", "nrhs", "nb", "waves", "xcd_map", "passes", "lds_kb", "ms"}, ...]} (created when absent), one
 * entry per line; the key is the device (architecture name and compute-unit count),
 * the lattice extents and the FP32 link storage ("link12" / "link18").  The call sets
 * every cached tile of the lattice's key for a right-hand-side count the lattice has
 * no tile for yet, then writes the lattice's tiles (tuned or set, with the tuner's
 * time where known) back under its key, keeping the other keys' entries; the file
 * is replaced through a temporary file.  Timing is left to ddq_tune_multi_rhs: a
 * first run tunes and saves, later runs load.  DDQ_ERR_ARG when the file cannot be
 * written or holds an invalid tile for this key. */
int ddq_autotune(ddq_lattice* lat, const char* cache_json_path);

/* |lambda_max(D_S)| by power iteration in FP64 (Sect. 2.4.4):
 * out = (|D_S^iters v0| / |v0|)^(1/iters).  v0: FP64 parity vector (device,
 * not modified).  Synchronises the stream. */
int ddq_estimate_lambda_max(ddq_lattice* lat, int iters, const void* v0, double* out);

/* eq. 2, FP64: bt_e = b_e - D_eo D_oo^-1 b_o (b: full vector, bt_e: parity
 * vector) and x = (x_e, D_oo^-1 (b_o - D_oe x_e)) (x: full vector). */
int ddq_oe_prepare(ddq_lattice* lat, int nrhs, const void* b, void* bt_e);
int ddq_oe_reconstruct(ddq_lattice* lat, int nrhs, const void* x_e, const void* b, void* x);

/* Restarted GMRES(m) of Alg. 2 on D_S with eq. 2 around it, for nrhs systems
 * D x_r = b_r solved one after the other (ddq_batch_solve runs several in lock-step).
 *   m            cycle length (1 <= m <= 128)
 *   max_cycles   restarts before giving up (DDQ_NOT_CONVERGED)
 *   tol          the full residual |b - D x| <= tol * |b| (the fine-level tolerance
 *                of the paper's parameter table is 1e-10).  The restarts run until
 *                |b~_e - D_S x_e| <= tol |b|, the same in exact arithmetic; then x is
 *                reconstructed (eq. 2) and |b - D x| formed in FP64 (eq. 1 on both
 *                parities); if rounding left it above tol |b|, the Schur target is
 *                lowered by the observed ratio and the restarts continue
 *   inner_prec   DDQ_F64: every operator apply in FP64.  DDQ_F32: inside a cycle
 *                the operator and the smoother run in FP32 on FP64 Arnoldi
 *                vectors (iterative refinement: the residual at every restart,
 *                the orthogonalisation and the update are FP64)
 *   smoother_sweeps  nu > 0: right preconditioner z = M v of nu Richardson
 *                sweeps from zero (flexible GMRES); 0: none
 *   omega        Richardson weight of the preconditioner
 *   inner_reduction  a cycle ends once its residual estimate has fallen by
 *                this factor (0 = automatic: 0 for FP64, 1e-5 for FP32)
 *   smoother_prec  DDQ_F16 / DDQ_BF16: the preconditioner's Richardson sweeps
 *                run on 16-bit storage (inner_prec must be DDQ_F32, the lattice
 *                must hold 16-bit links: DDQ_STORE_F16 / DDQ_STORE_BF16); the
 *                basis vector is scaled by sqrt(12 V/2) on the way in and back on
 *                the way out (the sweeps are linear); any other value: the
 *                sweeps run in inner_prec
 *   cycle_graph  (ddq_batch_solve only) nonzero: every restart cycle runs exactly
 *                m Arnoldi steps as one HIP graph launch, the basis normalisation
 *                computed on the device, and the host reads every step's
 *                coefficients once per cycle, keeping per system the columns up to
 *                the first whose estimate meets the cycle target (the steps after it
 *                are spent); 0: one graph and one host synchronisation per step,
 *                each system leaving the cycle when its estimate meets the target
 *   orth_passes  classical Gram-Schmidt passes per Arnoldi step: 2 (CGS2, the
 *                default; 0 means 2) or 1 (one pass: half the reads of the basis;
 *                enough where the cycle's own target, 1e-5 with an FP32 operator,
 *                lies far above the FP64 loss of orthogonality)
 * x: nrhs full vectors [nrhs][t][z][y][x][4][3], in the initial guesses, out the
 * solutions; b: nrhs full vectors; both complex128, not overlapping.  info (may be
 * NULL) receives one record per right-hand side: counts and the final full residual
 * (FP64, recomputed).  Work space: DDQ_RESERVE_SOLVE of ddq_reserve with max_m >= m
 * (else DDQ_ERR_STATE).  Returns DDQ_NOT_CONVERGED when any system missed tol.
 * Synchronises the stream. */
typedef struct {
  int m;
  int max_cycles;
  double tol;
  int inner_prec;
  int smoother_sweeps;
  double omega;
  double inner_reduction;
  int smoother_prec;
  int orth_passes;
  int cycle_graph;
} ddq_gmres_params;

typedef struct {
  int cycles;            /* restarts performed */
  int iters;             /* Arnoldi steps */
  int applies_f64;       /* D_S applications in FP64 (smoother sweeps included) */
  int applies_lo;        /* D_S applications in FP32 (smoother sweeps included) */
  double true_relres;    /* |b - D x| / |b|, FP64, recomputed after the last update */
  double t_total_ms;     /* wall time of the call */
} ddq_solve_info;

int ddq_oe_gmres_solve(ddq_lattice* lat, int nrhs, void* x, const void* b,
                       const ddq_gmres_params* params, ddq_solve_info* info);

/* The full Wilson-clover operator D of eq. 1 (nine 12x12 blocks per block row, Sect.
 * 2.3): y = D x for nrhs full FP64 vectors (the layout of ddq_pack_parity's full
 * vectors).  Kernel B's apply mode on each parity: y_e = A_ee x_e - H_eo x_o and
 * y_o = A_oo x_o - H_oe x_e, with the undivided odd clover blocks A_oo that
 * ddq_set_clover keeps for this.  x, y: device, not overlapping.  Work space: 8 FP64
 * parity vectors per right-hand side (DDQ_RESERVE_FULL of ddq_reserve). */
int ddq_apply_dirac(ddq_lattice* lat, int nrhs, const void* x, void* y);

/* The odd-even smoother M_nu of Sect. 2.4.5 (the right panel of Fig. 1): z = M_nu r for
 * nrhs full FP64 vectors, eq. 2's factorised D^-1 with D_S^-1 replaced by the
 * Richardson polynomial p_{R,nu}(D_S) = (I - (I - omega D_S)^nu) D_S^-1 of Sect. 2.4.4:
 * b~_e = b_e - D_eo D_oo^-1 r_o, x_e = nsweeps Richardson sweeps (Alg. 4) on D_S x_e = b~_e
 * from zero, z = (x_e, D_oo^-1 (r_o - D_oe x_e)).  prec: DDQ_F64, or DDQ_F32 for the
 * sweeps (FP32 storage and arithmetic; prepare and reconstruct stay FP64).  nsweeps = 0
 * gives z = (0, D_oo^-1 r_o).  r, z: device, not overlapping.  Work space as
 * ddq_apply_dirac, plus 2 FP32 parity vectors per right-hand side for DDQ_F32. */
int ddq_oe_smoother(ddq_lattice* lat, int nrhs, const void* r, void* z, int nsweeps, double omega, int prec);

/* SAP(n, m) of Alg. 1 (Sect. 2.4.1) on D x = b, FP64 full vectors, as a smoother: n
 * sweeps, each over the red then the black blocks, every block solve from the residual
 * b - D x recomputed before its colour (the listing's convergence exit is left out:
 * exactly n sweeps).  Blocks are 4^4, aligned at the origin (every lattice extent a
 * multiple of 4, else DDQ_ERR_ARG); a block's colour is the parity of the sum of its
 * block coordinates (with an odd number of blocks along a direction, the blocks on
 * either side of that boundary share a colour).  Block system: D restricted to the
 * block's sites (hops that leave it dropped; a block that spans a whole direction keeps
 * its wrap-around hops, with the antiperiodic sign in t), solved approximately by
 * odd-even preconditioning on the block and m Minimal Residual steps on the block's
 * Schur complement from zero, then added to x on the block.  prec: the block solves in
 * DDQ_F64, or in DDQ_F32 with the FP32 links (12-real if stored so) and clover blocks
 * (their dot products accumulated in FP64); the residuals b - D x and the update of x
 * are FP64 either way; a colour's residual is computed on that colour's blocks only (the
 * sites its block solves read).  x: initial guess in, iterate out; b: right-hand side
 * (device, not overlapping).  One workgroup per block, the block's half vectors in LDS
 * (FP32 with 12-real links: also the block's links).  Work space: DDQ_RESERVE_SAP of
 * ddq_reserve (the links and clover blocks of the block solves, and the FP64 links and
 * clover blocks of the residual, are copied into SAP block order there on the first
 * call after ddq_set_gauge / ddq_set_clover).
 * Synchronises the stream. */
int ddq_sap_smooth(ddq_lattice* lat, int prec, void* x, const void* b, int n, int m);

/* Flexible GMRES(m) of Alg. 2 on the full D x = b (FP64 full vectors; the fine-level
 * solver of Sect. 2.3) with M_nu (ddq_oe_smoother) as right preconditioner: nu =
 * params->smoother_sweeps, omega = params->omega, the sweeps in params->inner_prec
 * (DDQ_F64 or DDQ_F32; params->smoother_prec must be 0 or equal to it).  The
 * Gram-Schmidt passes and the stopping rule are those of ddq_oe_gmres_solve: |b - D x|
 * <= tol |b| on the FP64 residual recomputed at a restart; inner_reduction > 0 ends a
 * cycle once its residual estimate has fallen by that factor (0: at the target).
 * cycle_graph is ignored.  x: initial guess in, solution out (device).  Work space:
 * 2m + 2 full FP64 vectors plus the smoother's (DDQ_RESERVE_FULL of ddq_reserve with
 * max_m >= m; DDQ_RESERVE_SAP for the SAP form below).  Returns DDQ_NOT_CONVERGED when
 * max_cycles restarts did not reach the target (x holds the last iterate). */
int ddq_fgmres_solve(ddq_lattice* lat, void* x, const void* b, const ddq_gmres_params* params,
                     ddq_solve_info* info);

/* The same FGMRES on the full D with SAP(sap_n, sap_m) (ddq_sap_smooth, from a zero
 * initial guess, block solves in params->inner_prec) as the right preconditioner:
 * z_k = SAP applied to D z = v_k.  The other smoother fields of params are not used;
 * the lattice extents must be multiples of 4.
 * applies_f64 counts the D applies of the Arnoldi steps and residuals. */
int ddq_fgmres_sap_solve(ddq_lattice* lat, void* x, const void* b, const ddq_gmres_params* params, int sap_n,
                         int sap_m, ddq_solve_info* info);

/* Batched solves: several lattices of different extents, several right-hand
 * sides each, all solved to their own tolerance in one call.  Each (lattice,
 * right-hand side) pair is one system x = D^-1 b treated exactly as by
 * ddq_oe_gmres_solve with inner_prec = DDQ_F32 (eq. 2 around the flexible,
 * mixed-precision GMRES(m) of Alg. 2 with the Richardson preconditioner of
 * Alg. 4); the paper solves one system at a time, the batching is this
 * library's.  All systems advance in lock-step: every Arnoldi step is one
 * replay of a HIP graph holding, for every lattice, the normalisation of v_k,
 * the nu FP32 Richardson sweeps and the FP32 D_S apply on all its right-hand
 * sides at once (the multi-right-hand-side kernels) and the FP64 classical
 * Gram-Schmidt (two passes) with the norms; the host then applies the Givens
 * rotations of every system after one synchronisation.  A system that has met
 * its cycle target idles on zero vectors until the slowest one finishes the
 * cycle; every cycle starts with FP64 residuals of all systems.
 *
 * ddq_batch_create: lats[nlat] distinct lattice handles, each with FP64 and FP32
 *   links (ddq_set_gauge) and clover (ddq_set_clover); nrhs[l] >= 1 right-hand
 *   sides for lattice l.  The batch keeps the handles (destroy it before them) and
 *   owns its own stream (default priority) and work buffers.
 *   hip_stream: the caller's stream; a solve starts after the work enqueued on it.
 * ddq_batch_reserve: allocates the batch's work space for cycle lengths up to max_m
 *   (1 .. 127; cycle_graph != 0 adds the cycle mode's coefficient arrays): per
 *   lattice (2 max_m + 5) FP64 and 3 FP32 batched parity vectors, u_o of nrhs[l]
 *   right-hand sides in every precision the lattice stores, the pinned host
 *   buffers; and tunes (ddq_tune_multi_rhs) every lattice with no tile for its
 *   count.  Synchronises.  A solve needs it (else DDQ_ERR_STATE) and allocates
 *   nothing.
 * ddq_batch_solve: x[l], b[l] complex128 full vectors [nrhs[l]][t][z][y][x][4][3]
 *   on the device (x in: initial guess, out: solution; b not modified).  params as
 *   for ddq_oe_gmres_solve (m <= 127, inner_prec must be DDQ_F32); omegas[l] (or
 *   NULL: params->omega for all) the Richardson weight of lattice l.  info (may be
 *   NULL) receives one record per system in (lattice, right-hand side) order; the
 *   counts are those of the lock-step run.  The stopping rule is that of
 *   ddq_oe_gmres_solve: after the restarts have brought every system to
 *   |b~_e - D_S x_e| <= tol |b|, its full residual |b - D x| is formed in FP64 and a
 *   system above tol |b| continues with a lowered Schur target.  Synchronises;
 *   returns DDQ_OK when every system met |b - D x| <= tol |b|, DDQ_NOT_CONVERGED
 *   otherwise.
 *   Graphs are captured on the first solve and again when m, nu, an omega or a
 *   lattice's buffers change.  One thread at a time per batch; a lattice in a
 *   batch must not be used by other calls while a batch solve runs. */
typedef struct ddq_batch ddq_batch;

int ddq_batch_create(ddq_lattice* const* lats, const int* nrhs, int nlat, void* hip_stream, ddq_batch** out);
int ddq_batch_reserve(ddq_batch* batch, int max_m, int cycle_graph);
int ddq_batch_solve(ddq_batch* batch, void* const* x, const void* const* b, const ddq_gmres_params* params,
                    const double* omegas, ddq_solve_info* info);
int ddq_batch_destroy(ddq_batch* batch);

/* Backward pass of y_e = D_S(U) x_e (pattern: differentiation).
 * ddq_backward_apply: grad_x_e = D_S^H grad_y_e = g5 D_S g5 grad_y_e (the adjoint
 *   apply; the same as ddq_apply_schur with dagger = 1).
 * ddq_backward_link_force: for L = Re(chi_e^H D_S(U) phi_e) (chi_e the upstream
 *   gradient of y_e), the derivative with respect to every link, FP64:
 *     G  complex128 [t][z][y][x][mu][3][3]: dL = Re tr(G^H dU) (torch's convention
 *        for the gradient of a real function of complex U), or NULL;
 *     F  double [t][z][y][x][mu][8]: F_a = dL/de for U -> exp(i e T_a) U,
 *        T_a = lambda_a / 2, i.e. F_a = -Im tr(T_a U G^H), or NULL.
 *   Both the hopping term and the clover term (its leaves and the inverse A_oo^-1)
 *   are differentiated.  accumulate != 0 adds to G / F instead of overwriting.
 *   chi_e, phi_e: FP64 parity vectors.  Needs the canonical links set by
 *   ddq_set_gauge and the clover of ddq_set_clover.  Work space (two parity
 *   vectors and V x 54 complex128 insertions): DDQ_RESERVE_FORCE of ddq_reserve. */
int ddq_backward_apply(ddq_lattice* lat, int prec, int nrhs, const void* grad_y_e, void* grad_x_e);
int ddq_backward_link_force(ddq_lattice* lat, const void* chi_e, const void* phi_e, void* G, void* F,
                            int accumulate);

/* Per-kernel timing of the stencil kernels.  Between ddq_profile_begin and
 * ddq_profile_end every stencil launch on the lattice's stream is bracketed by
 * two HIP events on that stream.  ddq_profile_end synchronises the stream and
 * fills up to max_entries records, one per kernel variant, with the launch count,
 * the summed event time and the kernel's algorithmic bytes per launch (every
 * field touched once per launch: links, clover blocks and spinors; the roofline
 * numerator).  *n_out receives the number of variants seen. */
typedef struct {
  char name[40];
  int launches;
  double total_ms;
  double bytes_per_launch;
} ddq_kernel_stats;

int ddq_profile_begin(ddq_lattice* lat);
int ddq_profile_end(ddq_lattice* lat, ddq_kernel_stats* out, int max_entries, int* n_out);

/* STREAM-style device copy of `bytes` (a multiple of 16) from src to dst on
 * hip_stream, one 16-byte element per thread: the attainable-bandwidth probe
 * reported next to the HBM peak, and (plain form) the calibration kernel of the
 * traffic counters.  nontemporal != 0 reads and writes with the non-temporal
 * cache policy.  dst and src are device pointers, 16-byte aligned, not
 * overlapping. */
int ddq_stream_copy(void* dst, const void* src, int64_t bytes, int nontemporal, void* hip_stream);

/* Streaming ceiling of a one-right-hand-side stencil kernel: a measurement aid
 * reported next to the HBM peak, not part of the operator.  For every site it moves
 * the bytes that kernel moves once per site -- the input spinor (the site's own rows
 * in place of its eight neighbours'), the four link fields and the clover field of
 * the lattice's `prec` storage (12-real FP32 links if stored so), x and b where the
 * kernel reads them, the output rows -- with the same layouts, workgroup order and
 * cache policies, combined without arithmetic: the rate the memory system delivers
 * for the kernel's byte mix without its neighbour gathers.
 *   kernel  0: A (in -> out, odd links and clover), 1: B apply (in, x -> out),
 *           2: B Richardson (in, x, b -> out; even links and clover)
 *   prec    DDQ_F32 or DDQ_F64; in, x, b, out: parity vectors of that precision on
 *           the lattice's device (x, b may be NULL where unread; out receives
 *           meaningless values and must not overlap the others)
 * Launched on the lattice's stream; profiled as stream_<kernel name> when
 * profiling is on (the same algorithmic bytes as the stencil kernel). */
int ddq_stencil_stream(ddq_lattice* lat, int prec, int kernel, const void* in, const void* x, const void* b,
                       void* out);

/* Coarse-grid operator of the two-level method (Sect. 2.3): the Galerkin operator
 * D_c = P^H D P of an aggregation-based prolongation P is nearest-neighbour on the
 * coarse lattice, with nine dense 2N_v x 2N_v complex blocks per coarse site, so
 *     y(x) = sum_{d=0..8} A(x, d) v(x + d)
 * with d = 0 the site's own block and d = 1 + 2 mu + s the block coupling to the
 * neighbour in direction mu (0..3 = x, y, z, t), forward (s = 0) or backward (s = 1).
 * The coarse lattice is periodic in all directions (a fine antiperiodic boundary sign
 * is part of the blocks).  Coarse site index x + Cx*(y + Cy*(z + Cz*t)); a coarse
 * vector row q in 0 .. 2N_v-1 is chirality q / N_v, test vector q % N_v.  Blocks are
 * stored in FP32 (Sect. 3.3 applies them in single precision) or, with `storage` =
 * DDQ_F16 / DDQ_BF16, in 16 bits (the lower coarse-level precision the paper leaves to
 * future work: half the block bytes; FP16 rounds once from the caller's values, BF16
 * through FP32; FP16's range is the caller's to respect), and applied with FP32
 * arithmetic and accumulation on the matrix cores; the library does not build P or the
 * blocks.
 *
 * ddq_coarse_packed_bytes: bytes of the packed block array for coarse extents cdims
 *   (each >= 1, at most 2^25 sites), N_v test vectors (1 .. 32) and a storage.
 * ddq_coarse_pack_blocks: converts blocks[site][d][row i][column k] (row-major complex
 *   numbers, complex128 for prec = DDQ_F64 or complex64 for DDQ_F32) into the apply's
 *   packed operand order in the given storage (zero-padded to 16 x 8 tiles) in `packed`, a caller-owned
 *   device array of ddq_coarse_packed_bytes bytes, 16-byte aligned.  Enqueued on
 *   hip_stream; allocates nothing.
 * ddq_coarse_apply: y = D_c v for nrhs right-hand sides (1 .. 1048560); v and y are
 *   complex64 device arrays [site][row 2N_v][rhs nrhs] (right-hand side innermost), and
 *   `packed` the blocks as ddq_coarse_pack_blocks left them in the same storage,
 *   8-byte aligned, y not overlapping v.  One wavefront per coarse site and per group of
 *   rhs_tiles_per_wave tiles of 16 right-hand sides (1 .. 4; 0 = the default: the fewest
 *   groups of at most 4 tiles, of balanced size); every group reads the packed blocks once,
 *   and up to four groups of one site run in one workgroup, sharing them through the caches.
 *   product: how a complex product is formed on the matrix cores: 1 = four real products
 *   (Re = ArVr - AiVi, Im = ArVi + AiVr), 2 = Gauss's three (P = Ar(Vr + Vi),
 *   Q = (Ar + Ai)Vi, R = (Ai - Ar)Vr; Re = P - Q, Im = P + R: a quarter fewer products, the
 *   sums rounded to FP32 first), 0 = the default (three).  Both stay within a small
 *   multiple of 2^-24 x sum |A||v| per output element.  Enqueued on hip_stream; allocates nothing.
 * Errors: DDQ_ERR_ARG for null or misaligned pointers and sizes out of range,
 * DDQ_ERR_HIP if a launch fails. */
int ddq_coarse_packed_bytes(const int cdims[4], int nv, int storage, int64_t* bytes);
int ddq_coarse_pack_blocks(const int cdims[4], int nv, int storage, int prec, const void* blocks, void* packed,
                           void* hip_stream);
int ddq_coarse_apply(const int cdims[4], int nv, int storage, int nrhs, const void* packed, const void* v, void* y,
                     int rhs_tiles_per_wave, int product, void* hip_stream);

/* Thread-local message of the last error (empty string if none). */
const char* ddq_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DDQ_H */
