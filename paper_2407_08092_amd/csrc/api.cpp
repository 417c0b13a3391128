// api.cpp -- the C ABI (include/ddq.h): lattice handles, set-up, operator
// applications, Richardson smoothing, power iteration, eq. 2 prepare /
// reconstruct and the restarted (flexible, mixed-precision) GMRES of Alg. 2.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <complex>
#include <cstdio>
#include <cstring>
#include <string>
#include <functional>
#include <mutex>
#include <vector>

#include "../../include/ddq.h"
#include "ddq_internal.h"
#include "coarse_internal.h"

using namespace ddq;
using cd = std::complex<double>;

namespace {

thread_local std::string g_err;

int fail(int code, const std::string& msg) {
  g_err = msg;
  return code;
}

#define HIPCHK(expr)                                                                  \
  do {                                                                                \
    hipError_t e_ = (expr);                                                           \
    if (e_ != hipSuccess)                                                             \
      return fail(DDQ_ERR_HIP, std::string(#expr) + " failed: " + hipGetErrorString(e_)); \
  } while (0)

#define CHK(expr)            \
  do {                       \
    int r_ = (expr);         \
    if (r_ < 0) return r_;   \
  } while (0)

int dalloc(void** p, size_t bytes) {
  *p = nullptr;
  if (bytes == 0) return DDQ_OK;
  hipError_t e = hipMalloc(p, bytes);
  if (e != hipSuccess) {
    *p = nullptr;
    (void)hipGetLastError();
    return fail(e == hipErrorOutOfMemory ? DDQ_ERR_OOM : DDQ_ERR_HIP,
                "hipMalloc of " + std::to_string(bytes) + " bytes failed: " + hipGetErrorString(e));
  }
  return DDQ_OK;
}

void dfree(void*& p) {
  if (p) (void)hipFree(p);
  p = nullptr;
}

// Work space is allocated only by the calls that own it (lattice creation, the set-up
// calls, the reservations and the tuner); they open an AllocScope.  Everywhere else a
// buffer that is too small is an error: apply, smooth and solve calls allocate nothing.
thread_local int g_alloc_depth = 0;
struct AllocScope {
  AllocScope() { ++g_alloc_depth; }
  ~AllocScope() { --g_alloc_depth; }
};

// a device buffer that only grows
struct Grow {
  void* p = nullptr;
  size_t bytes = 0;
  int ensure(size_t need) {
    if (need <= bytes) return DDQ_OK;
    if (g_alloc_depth == 0)
      return fail(DDQ_ERR_STATE, "work space of " + std::to_string(need) + " bytes needed, " +
                                     std::to_string(bytes) + " reserved: call ddq_reserve (or ddq_batch_reserve) first");
    dfree(p);
    bytes = 0;
    int r = dalloc(&p, need);
    if (r == DDQ_OK) bytes = need;
    return r;
  }
  void release() {
    dfree(p);
    bytes = 0;
  }
};

// Fixed work space of ddq_apply_schur_noalloc: a file-scope device array, one copy per
// GPU, alive until the process ends.  Host code never passes the array's name to a
// kernel (on the host it is only a stand-in symbol); it uses the device address that
// hipGetSymbolAddress returns, looked up once per device by ddq_create_lattice with the
// lattice's device current.
constexpr size_t NOALLOC_SCRATCH_BYTES = size_t(64) << 20;
static __device__ __align__(256) unsigned char scratch[NOALLOC_SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;
std::mutex g_scratch_mu;
void* g_scratch_dev[MAX_DEVICES] = {};

// device address of `scratch` on the current device (resolved on first use)
int scratch_address(int* device, void** out) {
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev < 0 || dev >= MAX_DEVICES) return fail(DDQ_ERR_HIP, "device ordinal out of range");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_dev[dev]) {
    void* p = nullptr;
    HIPCHK(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return fail(DDQ_ERR_HIP, "hipGetSymbolAddress returned a null address for the work space");
    g_scratch_dev[dev] = p;
  }
  *device = dev;
  *out = g_scratch_dev[dev];
  return DDQ_OK;
}

// set while a call that must not allocate runs: the per-kernel profiler (which creates
// HIP events) stands aside
thread_local bool g_no_alloc_call = false;

}  // namespace

struct ddq_lattice {
  int dims[4];
  int anti;
  int64_t V, Vh;
  Geo geo;
  hipStream_t stream;
  // canonical FP64 links kept on the device for the clover build
  void* U = nullptr;
  bool have_gauge = false;
  unsigned store = 0;
  void* links[4][2] = {};  // [prec][parity]; FP16 / BF16 fields are 12-real
  void* clov[4][2] = {};   // [prec][0: A_ee, 1: A_oo^-1]
  void* clov_oo = nullptr;  // FP64 A_oo (undivided), for the full operator D
  bool have_clover = false;
  bool link12 = false;  // FP32 links stored as their first two rows
  double c_sw = 0.0, m0 = 0.0;
  // work buffers
  Grow force_ws;      // force: psi_o, lambda_o, insertions
  Grow tmp[4];        // u_o per precision
  Grow scratch64;     // FP64 parity vectors
  Grow scratch32;     // FP32 parity vectors
  Grow oe_ws64;       // full operator and odd-even smoother: FP64 parity vectors
  Grow oe_ws32;       // the smoother's FP32 parity vectors
  Grow sap_links[2], sap_clov[2];  // links and clover blocks per parity in SAP order
  int sap_prec = -1;               // their precision; -1: not built for the current fields
  Grow sap_rlinks[2], sap_rclov[2];  // FP64 links and A_ee, A_oo in SAP order (SAP residual)
  bool sap_res_ok = false;           // built for the current fields
  Grow partial;       // reduction partials
  Grow small;         // device scalars: h (2 x 256 complex), norms
  double* host = nullptr;  // pinned host mirror of `small`
  size_t host_bytes = 0;
  int nbx = 0;        // workgroups of the reduction kernels
  // the reservation of ddq_reserve (grown, never shrunk): right-hand sides, cycle length
  // and the DDQ_RESERVE_* call families whose work space is kept
  int res_nrhs = 1, res_m = 0;
  // the lattice's device and that device's copy of the fixed work space
  int device = -1;
  void* noalloc_ws = nullptr;
  unsigned res_what = 0;

  // per-kernel timing (ddq_profile_begin / ddq_profile_end)
  bool prof_on = false;
  std::vector<hipEvent_t> ev;          // pairs: start 2k, stop 2k+1
  std::vector<int> ev_kind;            // kind of pair k
  int ev_used = 0;
  std::vector<std::string> kind_name;
  std::vector<double> kind_ms, kind_bytes;
  std::vector<int> kind_n;

  // launch settings of the mrhs-layout stencil (ddq_mrhs_set_launch)
  int mrhs_order = MRHS_ORDER_SLAB, mrhs_lds_kb = 0, mrhs_tsteps = 0, mrhs_stage = 1;
  // the 16-bit stencil reads the FP32 clover blocks (ddq_set_h16_clover)
  bool h16_clover32 = false;
  // one-right-hand-side sweeps and applies on this many t-chunks (ddq_set_sweep_chunks;
  // 0: chosen from the lattice size)
  int sweep_chunks = 0;

  // FP32 multi-right-hand-side tiles by right-hand-side count (ddq_tune_multi_rhs)
  std::vector<std::pair<int, MrTile>> tiles;
  std::vector<std::pair<int, double>> tile_ms;  // the tuner's time of the chosen tile
  const MrTile* tile_for(int nrhs) const {
    for (const auto& t : tiles)
      if (t.first == nrhs) return &t.second;
    return nullptr;
  }

  long long nvec() const { return 12LL * Vh; }  // complex elements of one parity vector
};

namespace {

int check_lat(const ddq_lattice* L) {
  if (!L) return fail(DDQ_ERR_ARG, "null lattice handle");
  return DDQ_OK;
}

int check_prec(int prec) {
  if (prec != DDQ_F64 && prec != DDQ_F32 && prec != DDQ_F16 && prec != DDQ_BF16)
    return fail(DDQ_ERR_ARG, "precision must be DDQ_F64, DDQ_F32, DDQ_F16 or DDQ_BF16");
  return DDQ_OK;
}
bool is16(int prec) { return prec == DDQ_F16 || prec == DDQ_BF16; }
int h16_kind(int prec) { return prec == DDQ_BF16 ? H16_BF16 : H16_F16; }

int check_ready(const ddq_lattice* L, int prec) {
  CHK(check_lat(L));
  CHK(check_prec(prec));
  if (!L->have_gauge) return fail(DDQ_ERR_STATE, "ddq_set_gauge has not been called");
  if (!L->links[prec][0]) return fail(DDQ_ERR_STATE, "links not stored in the requested precision");
  if (!L->have_clover) return fail(DDQ_ERR_STATE, "ddq_set_clover has not been called");
  return DDQ_OK;
}

// bytes per stored complex number of a parity vector
size_t elem_bytes(int prec) { return prec == DDQ_F64 ? 16 : (prec == DDQ_F32 ? 8 : 4); }

int ensure_host(ddq_lattice* L, size_t bytes) {
  if (bytes <= L->host_bytes) return DDQ_OK;
  if (g_alloc_depth == 0) return fail(DDQ_ERR_STATE, "pinned host buffer too small");
  if (L->host) (void)hipHostFree(L->host);
  L->host = nullptr;
  L->host_bytes = 0;
  HIPCHK(hipHostMalloc((void**)&L->host, bytes, hipHostMallocDefault));
  L->host_bytes = bytes;
  return DDQ_OK;
}

// ---------------------------------------------------------------------------
// operator building blocks
// ---------------------------------------------------------------------------
// algorithmic bytes of one stencil launch: every field touched once
double hop_bytes(const ddq_lattice* L, int prec, int mode, int nrhs) {
  // complex numbers per site: spinor rows (12 each) per right-hand side, 72 link
  // entries (8 directions x 9), 36 clover pairs (2 blocks x 18 slots)
  int spin = 0;
  bool clover = true;
  switch (mode) {
    case M_HOP_CLINV: spin = 2; break;            // in, out
    case M_RECON: spin = 3; break;                // in, b, out
    case M_APPLY: spin = 3; break;                // in, x, out
    case M_RICH: spin = 4; break;                 // in, x, b, out
    case M_RESID: spin = 4; break;                // in, x, b, out
    case M_PREP: spin = 3; clover = false; break; // in, b, out
  }
  if (is16(prec)) {  // 12-real links, 4 bytes per complex; clover: 40 padded 16-bit slots or 36 FP32 pairs
    const double cl = !clover ? 0.0 : (L->h16_clover32 ? 36.0 * 8 : 40.0 * 4);
    return ((double)(12 * spin * nrhs + 48) * 4 + cl) * (double)L->Vh;
  }
  const int link = (prec == DDQ_F32 && L->link12) ? 48 : 72;
  const double per_site = (double)(12 * spin * nrhs + link + (clover ? 36 : 0)) * (prec == DDQ_F64 ? 16 : 8);
  return per_site * (double)L->Vh;
}

const char* mode_name(int mode) {
  static const char* n[] = {"hop_clinv", "hop_recon", "hop_apply", "hop_richardson", "hop_resid", "hop_prep"};
  return n[mode];
}

int prof_flush(ddq_lattice* L) {
  if (L->ev_used == 0) return DDQ_OK;
  HIPCHK(hipEventSynchronize(L->ev[2 * (L->ev_used - 1) + 1]));
  for (int k = 0; k < L->ev_used; ++k) {
    float ms = 0.f;
    HIPCHK(hipEventElapsedTime(&ms, L->ev[2 * k], L->ev[2 * k + 1]));
    L->kind_ms[L->ev_kind[k]] += ms;
    L->kind_n[L->ev_kind[k]] += 1;
  }
  L->ev_used = 0;
  return DDQ_OK;
}

// launch a stencil kernel, bracketed by events while profiling
// the multi-right-hand-side FP32 kernels take the lattice's tuned tile when one fits
template <typename R>
hipError_t launch_any(ddq_lattice* L, const HopArgs<R>& a, int mode, bool dag, int nrhs) {
  const MrTile* t = nrhs > 1 ? L->tile_for(nrhs) : nullptr;
  HopArgs<R> b = a;
  if constexpr (sizeof(R) == 4) {
    if (t && hop_rb_supported(mode, dag, nrhs, *t)) {
      b.tile = *t;
      return launch_hop_rb(b, mode, nrhs, L->stream);
    }
  }
  // one right-hand side per thread: the workgroup order of an nb = 0 tile set for
  // nrhs, else slab order
  b.tile = MrTile{};
  b.tile.xmap = (t && t->nb == 0) ? t->xmap : XMAP_SLAB;
  return launch_hop<R>(b, mode, dag, nrhs, L->stream);
}

// run `launch` bracketed by profiling events on the lattice's stream (when on),
// its time booked under `name` with `bytes` algorithmic bytes per launch
template <typename F>
hipError_t prof_launch(ddq_lattice* L, const std::string& name, double bytes, F launch) {
  if (!L->prof_on || g_no_alloc_call) return launch();
  int kind = -1;
  for (size_t k = 0; k < L->kind_name.size(); ++k)
    if (L->kind_name[k] == name) kind = (int)k;
  if (kind < 0) {
    kind = (int)L->kind_name.size();
    L->kind_name.push_back(name);
    L->kind_ms.push_back(0.0);
    L->kind_n.push_back(0);
    L->kind_bytes.push_back(0.0);
  }
  L->kind_bytes[kind] += bytes;  // summed over launches (chunked launches differ in size)
  if (L->ev_used * 2 == (int)L->ev.size()) {
    if (L->ev.size() < 2048) {
      hipEvent_t e0, e1;
      hipError_t e = hipEventCreate(&e0);
      if (e != hipSuccess) return e;
      e = hipEventCreate(&e1);
      if (e != hipSuccess) return e;
      L->ev.push_back(e0);
      L->ev.push_back(e1);
      L->ev_kind.push_back(0);
    } else if (prof_flush(L) != DDQ_OK) {
      return hipErrorUnknown;
    }
  }
  const int k = L->ev_used++;
  L->ev_kind[k] = kind;
  hipError_t e = hipEventRecord(L->ev[2 * k], L->stream);
  if (e != hipSuccess) return e;
  e = launch();
  if (e != hipSuccess) return e;
  return hipEventRecord(L->ev[2 * k + 1], L->stream);
}

// launch a stencil kernel, bracketed by events while profiling
template <typename R>
hipError_t run_hop(ddq_lattice* L, const HopArgs<R>& a, int mode, bool dag, int nrhs) {
  if (!L->prof_on || g_no_alloc_call) return launch_any<R>(L, a, mode, dag, nrhs);
  const int prec = sizeof(R) == 8 ? DDQ_F64 : DDQ_F32;
  std::string tile;
  if (prec == DDQ_F32 && nrhs > 1) {
    const MrTile* t = L->tile_for(nrhs);
    if (t && hop_rb_supported(mode, dag, nrhs, *t))
      tile = "_nb" + std::to_string(t->nb) + "g" + std::to_string(t->g) + (t->xmap ? "x" + std::to_string(t->xmap) : "") +
             (t->passes > 1 ? "p" + std::to_string(t->passes) : "") + (t->lds_kb ? "l" + std::to_string(t->lds_kb) : "");
  }
  std::string name = std::string(mode_name(mode)) + (prec == DDQ_F64 ? "_f64" : (a.link12 ? "_f32l12" : "_f32")) +
                     (dag ? "_dag" : "") + (nrhs > 1 ? "_x" + std::to_string(nrhs) : "") + tile;
  const double share = a.t_cnt > 0 ? (double)a.t_cnt / L->dims[3] : 1.0;  // a chunk of t-slices
  return prof_launch(L, name, hop_bytes(L, prec, mode, nrhs) * share,
                     [&]() { return launch_any<R>(L, a, mode, dag, nrhs); });
}

// the 16-bit-storage stencil: kernel A (M_HOP_CLINV) or kernel B (M_APPLY / M_RICH)
hipError_t run_hop16(ddq_lattice* L, int prec, int nrhs, int mode, const void* in, const void* x, const void* b,
                     void* out, float omega) {
  Hop16Args a{};
  const int p_out = mode == M_HOP_CLINV ? 1 : 0;
  a.g = L->geo;
  a.p_out = p_out;
  a.in = (const u4_t*)in;
  a.links = (const u4_t*)L->links[prec][p_out];
  a.clov = (const u4_t*)L->clov[prec][p_out];
  a.clov32 = L->h16_clover32 ? (const f2_t*)L->clov[DDQ_F32][p_out] : nullptr;
  a.x = (const u4_t*)x;
  a.b = (const u4_t*)b;
  a.out = (u4_t*)out;
  a.omega = omega;
  a.nrhs = nrhs;
  // workgroup order: that of the lattice's FP32 tile for this count, else slab order
  const MrTile* t = nrhs > 1 ? L->tile_for(nrhs) : nullptr;
  a.chunk = t ? t->xmap : XMAP_SLAB;
  if (!L->prof_on || g_no_alloc_call) return launch_hop16(h16_kind(prec), a, mode, L->stream);
  std::string name = std::string(mode_name(mode)) + (prec == DDQ_BF16 ? "_bf16" : "_f16") +
                     (L->h16_clover32 ? "_c32" : "") +
                     (nrhs > 1 ? "_x" + std::to_string(nrhs) : "");
  return prof_launch(L, name, hop_bytes(L, prec, mode, nrhs),
                     [&]() { return launch_hop16(h16_kind(prec), a, mode, L->stream); });
}

// u: work space for u_o (nrhs parity vectors of prec); null selects the lattice's own
int schur16(ddq_lattice* L, int prec, int nrhs, const void* x, void* y, void* u = nullptr) {
  if (!u) u = L->tmp[prec].p;
  HIPCHK(run_hop16(L, prec, nrhs, M_HOP_CLINV, x, nullptr, nullptr, u, 0.f));
  HIPCHK(run_hop16(L, prec, nrhs, M_APPLY, u, x, nullptr, y, 0.f));
  return DDQ_OK;
}

int sweeps16(ddq_lattice* L, int prec, int nrhs, void* x, const void* b, int n, float omega) {
  void* u = L->tmp[prec].p;
  for (int k = 0; k < n; ++k) {
    HIPCHK(run_hop16(L, prec, nrhs, M_HOP_CLINV, x, nullptr, nullptr, u, 0.f));
    HIPCHK(run_hop16(L, prec, nrhs, M_RICH, u, x, b, x, omega));
  }
  return DDQ_OK;
}

// the mrhs-layout stencil: kernel A (M_HOP_CLINV) or kernel B (M_APPLY / M_RICH), on the
// output sites of slices [t_lo, t_lo + t_cnt) when t_cnt > 0
hipError_t run_mrhs(ddq_lattice* L, int nrhs, int mode, int engine, const void* in, const void* x, const void* b,
                    void* out, float omega, int t_lo = 0, int t_cnt = 0) {
  MrhsArgs a{};
  const int p_out = mode == M_HOP_CLINV ? 1 : 0;
  a.g = L->geo;
  a.p_out = p_out;
  a.in = (const f2_t*)in;
  a.links = (const f2_t*)L->links[DDQ_F32][p_out];
  a.clov = (const f2_t*)L->clov[DDQ_F32][p_out];
  a.x = (const f2_t*)x;
  a.b = (const f2_t*)b;
  a.out = (f2_t*)out;
  a.omega = omega;
  a.link12 = L->link12 ? 1 : 0;
  a.nrhs = nrhs;
  a.engine = engine;
  a.order = L->mrhs_order;
  a.lds_kb = L->mrhs_lds_kb;
  a.tsteps = L->mrhs_order == MRHS_ORDER_TWALK ? L->mrhs_tsteps : 0;
  a.stage = L->mrhs_stage;
  a.t_lo = t_lo;
  a.t_cnt = t_cnt;
  if (!L->prof_on || g_no_alloc_call) return launch_hop_mrhs(a, mode, L->stream);
  std::string name = std::string(mode_name(mode)) + (a.link12 ? "_f32l12" : "_f32") + "_mrhs" +
                     std::to_string(nrhs) + (engine == MRHS_ENGINE_MFMA ? "_mfma" : "_valu") + (a.stage ? "_st" : "");
  const double share = t_cnt > 0 ? (double)t_cnt / L->dims[3] : 1.0;
  return prof_launch(L, name, hop_bytes(L, DDQ_F32, mode, nrhs) * share,
                     [&]() { return launch_hop_mrhs(a, mode, L->stream); });
}

template <typename R>
HopArgs<R> hop_args(const ddq_lattice* L, int prec, int p_out) {
  HopArgs<R> a{};
  a.g = L->geo;
  a.p_out = p_out;
  a.links = (const pair<R>*)L->links[prec][p_out];
  a.clov = (const pair<R>*)L->clov[prec][p_out];
  a.rhs_stride = L->nvec();
  a.link12 = (prec == DDQ_F32 && L->link12) ? 1 : 0;
  return a;
}

// u_o = A_oo^-1 H_oe x_e  (kernel A)
template <typename R>
hipError_t kernel_A(ddq_lattice* L, int prec, int nrhs, const pair<R>* x, pair<R>* u, bool dag) {
  HopArgs<R> a = hop_args<R>(L, prec, 1);
  a.in = x;
  a.out = u;
  return run_hop<R>(L, a, M_HOP_CLINV, dag, nrhs);
}

// even-side kernel B in one of its modes
template <typename R>
hipError_t kernel_B(ddq_lattice* L, int prec, int nrhs, int mode, const pair<R>* u, const pair<R>* x,
                    const pair<R>* b, pair<R>* out, R omega, bool dag) {
  HopArgs<R> a = hop_args<R>(L, prec, 0);
  a.in = u;
  a.x = x;
  a.b = b;
  a.out = out;
  a.omega = omega;
  return run_hop<R>(L, a, mode, dag, nrhs);
}

// Chunks of t-slices for the one-right-hand-side sweeps and applies: the number set by
// ddq_set_sweep_chunks, or (0, the default) for FP32 whose u_o (V/2 x 12 complex64) exceeds
// 128 MiB, enough chunks that one chunk's u_o stays near 40 MiB, a small part of the 256 MB
// Infinity Cache; else one launch.  Measured: 48^3 x 96 FP32 (509 MB of u_o) gains 5-7 %
// with 10-13 chunks; 48^3 x 12 (64 MB, cached anyway) loses 5 % with 2; FP64 at 48^3 x 96
// with 25 chunks is 1 % slower than one launch.
int chunks_for(const ddq_lattice* L, int prec) {
  int nc = L->sweep_chunks;
  if (nc == 0) {
    const double u_bytes = (double)L->nvec() * 8.0;
    nc = (prec == DDQ_F32 && u_bytes > 128.0 * 1024 * 1024) ? (int)std::ceil(u_bytes / (40.0 * 1024 * 1024)) : 1;
  }
  return std::max(1, std::min(nc, L->dims[3]));
}

// One Richardson sweep (mode M_RICH: out = x in place) or Schur apply (M_APPLY: out = y) on
// t-chunks: kernels A and B on the output sites of nc ranges of t-slices, ordered so that
// every B reads only u_o of the old x and every A reads x before the B of the chunk next to
// it updates it: A(nc-1), A(0), then per chunk c: A(c+1), B(c).  u_o of a chunk is read by
// its B one launch after its A wrote it.
template <typename R>
int sweep_chunked(ddq_lattice* L, int prec, const pair<R>* x, const pair<R>* b, pair<R>* u, pair<R>* out, R omega,
                  int nc, int mode, bool dag) {
  const int lt = L->dims[3];
  auto lo = [&](int c) { return (int)((long long)c * lt / nc); };
  auto runA = [&](int c) -> hipError_t {
    HopArgs<R> a = hop_args<R>(L, prec, 1);
    a.in = x;
    a.out = u;
    a.t_lo = lo(c);
    a.t_cnt = lo(c + 1) - lo(c);
    return run_hop<R>(L, a, M_HOP_CLINV, dag, 1);
  };
  auto runB = [&](int c) -> hipError_t {
    HopArgs<R> a = hop_args<R>(L, prec, 0);
    a.in = u;
    a.x = x;
    a.b = b;
    a.out = out;
    a.omega = omega;
    a.t_lo = lo(c);
    a.t_cnt = lo(c + 1) - lo(c);
    return run_hop<R>(L, a, mode, dag, 1);
  };
  HIPCHK(runA(nc - 1));
  HIPCHK(runA(0));
  for (int c = 0; c + 1 < nc; ++c) {
    if (c + 1 < nc - 1) HIPCHK(runA(c + 1));
    HIPCHK(runB(c));
  }
  HIPCHK(runB(nc - 1));
  return DDQ_OK;
}

// u: work space for u_o (nrhs parity vectors of prec); null selects the lattice's own
template <typename R>
int schur(ddq_lattice* L, int prec, int nrhs, const pair<R>* x, pair<R>* y, bool dag, pair<R>* u = nullptr) {
  if (!u) u = (pair<R>*)L->tmp[prec].p;
  const int nc = nrhs == 1 ? chunks_for(L, prec) : 1;
  if (nc > 1) return sweep_chunked<R>(L, prec, x, nullptr, u, y, R(0), nc, M_APPLY, dag);
  HIPCHK(kernel_A<R>(L, prec, nrhs, x, u, dag));
  HIPCHK(kernel_B<R>(L, prec, nrhs, M_APPLY, u, x, nullptr, y, R(0), dag));
  return DDQ_OK;
}

template <typename R>
int resid(ddq_lattice* L, int prec, int nrhs, const pair<R>* x, const pair<R>* b, pair<R>* r) {
  pair<R>* u = (pair<R>*)L->tmp[prec].p;
  HIPCHK(kernel_A<R>(L, prec, nrhs, x, u, false));
  HIPCHK(kernel_B<R>(L, prec, nrhs, M_RESID, u, x, b, r, R(0), false));
  return DDQ_OK;
}

template <typename R>
int sweeps(ddq_lattice* L, int prec, int nrhs, pair<R>* x, const pair<R>* b, int n, R omega) {
  pair<R>* u = (pair<R>*)L->tmp[prec].p;
  const int nc = chunks_for(L, prec);
  for (int k = 0; k < n; ++k) {
    if (nrhs == 1 && nc > 1) {
      CHK(sweep_chunked<R>(L, prec, x, b, u, x, omega, nc, M_RICH, false));
      continue;
    }
    HIPCHK(kernel_A<R>(L, prec, nrhs, x, u, false));
    HIPCHK(kernel_B<R>(L, prec, nrhs, M_RICH, u, x, b, x, omega, false));
  }
  return DDQ_OK;
}

int ensure_tmp(ddq_lattice* L, int prec, int nrhs) {
  return L->tmp[prec].ensure((size_t)nrhs * L->nvec() * elem_bytes(prec));
}

// Allocates the work space of the lattice's reservation (L->res_*) for the precisions
// it stores; called with an AllocScope open by ddq_reserve and the set-up calls.
//   every call: u_o of res_nrhs right-hand sides per stored precision; 2 res_nrhs FP64
//     parity vectors (prepare, reconstruct, power iteration)
//   SOLVE: ddq_oe_gmres_solve with m = res_m, one right-hand side at a time: 2m + 4 FP64
//     and 3 FP32 parity vectors
//   FULL: ddq_apply_dirac / ddq_oe_smoother on res_nrhs vectors (8 FP64 and 2 FP32 parity
//     vectors each), ddq_fgmres_solve (2m + 2 full FP64 vectors)
//   SAP: the SAP-ordered copies of links and clover, the residual work space, FGMRES
//   FORCE: the link force's insertions and two parity vectors
int reserve_impl(ddq_lattice* L) {
  const int nr = L->res_nrhs, m = L->res_m;
  const unsigned what = L->res_what;
  const size_t nv = (size_t)L->nvec();
  for (int prec = 0; prec < 4; ++prec)
    if (L->links[prec][0]) CHK(ensure_tmp(L, prec, nr));
  size_t n64 = 2 * (size_t)nr;
  if (what & DDQ_RESERVE_SOLVE) n64 = std::max(n64, (size_t)(2 * m + 4));
  if ((what & (DDQ_RESERVE_FULL | DDQ_RESERVE_SAP)) && m > 0) n64 = std::max(n64, (size_t)(4 * m + 4));
  CHK(L->scratch64.ensure(n64 * nv * 16));
  const bool f32 = L->links[DDQ_F32][0] != nullptr;
  if ((what & DDQ_RESERVE_SOLVE) && f32) CHK(L->scratch32.ensure(3 * nv * 8));
  if (what & (DDQ_RESERVE_FULL | DDQ_RESERVE_SAP)) {
    const size_t k = (what & DDQ_RESERVE_FULL) ? (size_t)nr : 1;
    CHK(L->oe_ws64.ensure(8 * k * nv * 16));
    if (f32 && (what & DDQ_RESERVE_FULL)) CHK(L->oe_ws32.ensure(2 * k * nv * 8));
  }
  if (what & DDQ_RESERVE_SAP) {
    const size_t fvh = (size_t)field_vh((int)L->Vh);
    for (int q = 0; q < 2; ++q) {  // the FP64 sizes cover the FP32 copies
      CHK(L->sap_links[q].ensure(4 * (size_t)LINK_ROWS * fvh * 16));
      CHK(L->sap_clov[q].ensure((size_t)CLOVER_ROWS * fvh * 16));
      CHK(L->sap_rlinks[q].ensure(4 * (size_t)LINK_ROWS * fvh * 16));
      CHK(L->sap_rclov[q].ensure((size_t)CLOVER_ROWS * fvh * 16));
    }
  }
  if (what & DDQ_RESERVE_FORCE) CHK(L->force_ws.ensure((2 * nv + (size_t)L->V * 54) * 16));
  return DDQ_OK;
}

// |v|^2 of n complex128 elements into device scalar dst
int norm2_dev(ddq_lattice* L, const d2_t* v, long long n, double* dst) {
  HIPCHK(launch_norm2_partial(v, n, (double*)L->partial.p, L->nbx, L->stream));
  HIPCHK(launch_reduce_real((const double*)L->partial.p, L->nbx, dst, L->stream));
  return DDQ_OK;
}

int fetch(ddq_lattice* L, const void* dev, size_t bytes) {
  CHK(ensure_host(L, bytes));
  HIPCHK(hipMemcpyAsync(L->host, dev, bytes, hipMemcpyDeviceToHost, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  return DDQ_OK;
}

int norm_host(ddq_lattice* L, const d2_t* v, long long n, double* out) {
  double* d = (double*)L->small.p;
  CHK(norm2_dev(L, v, n, d));
  CHK(fetch(L, d, sizeof(double)));
  *out = std::sqrt(L->host[0]);
  return DDQ_OK;
}

// eq. 2: b~_e = b_e - D_eo D_oo^-1 b_o = b_e + H_eo (A_oo^-1 b_o); bo: work vector(s)
int prepare_impl(ddq_lattice* L, int nrhs, const d2_t* b, d2_t* bt_e, d2_t* bo) {
  CHK(ensure_tmp(L, DDQ_F64, nrhs));
  d2_t* u = (d2_t*)L->tmp[DDQ_F64].p;
  HIPCHK(launch_pack_parity<double>(L->geo, 1, nrhs, b, bo, L->stream));
  HIPCHK(launch_clover_only<double>(L->geo, nrhs, (const d2_t*)L->clov[DDQ_F64][1], bo, u, L->stream));
  HIPCHK(launch_pack_parity<double>(L->geo, 0, nrhs, b, bt_e, L->stream));
  HIPCHK(kernel_B<double>(L, DDQ_F64, nrhs, M_PREP, u, nullptr, bt_e, bt_e, 0.0, false));
  return DDQ_OK;
}

// eq. 2: x_o = D_oo^-1 (b_o - D_oe x_e) = A_oo^-1 (b_o + H_oe x_e); bo, xo: work vectors
int reconstruct_impl(ddq_lattice* L, int nrhs, const d2_t* x_e, const d2_t* b, d2_t* x, d2_t* bo, d2_t* xo) {
  HIPCHK(launch_pack_parity<double>(L->geo, 1, nrhs, b, bo, L->stream));
  HopArgs<double> a = hop_args<double>(L, DDQ_F64, 1);
  a.in = x_e;
  a.b = bo;
  a.out = xo;
  HIPCHK(run_hop<double>(L, a, M_RECON, false, nrhs));
  HIPCHK(launch_unpack_parity<double>(L->geo, 0, nrhs, x_e, x, L->stream));
  HIPCHK(launch_unpack_parity<double>(L->geo, 1, nrhs, xo, x, L->stream));
  return DDQ_OK;
}

}  // namespace

// ===========================================================================
// C ABI
// ===========================================================================
extern "C" {

const char* ddq_last_error(void) { return g_err.c_str(); }

int ddq_create_lattice(const int dims[4], int t_antiperiodic, void* hip_stream, ddq_lattice** out) {
  if (!out) return fail(DDQ_ERR_ARG, "out is null");
  *out = nullptr;
  if (!dims) return fail(DDQ_ERR_ARG, "dims is null");
  long long V = 1;
  for (int k = 0; k < 4; ++k) {
    if (dims[k] < 2 || (dims[k] & 1))
      return fail(DDQ_ERR_ARG, "every extent must be even and >= 2 (got " + std::to_string(dims[k]) + ")");
    V *= dims[k];
  }
  if (V >= (1LL << 31)) return fail(DDQ_ERR_ARG, "volume must be below 2^31 sites");
  // every field is addressed through buffer descriptors of at most 2^32 - 1 bytes; the
  // largest one is the FP64 clover field of a parity (36 element rows of 16 bytes a site)
  if ((uint64_t)field_vh((int)(V / 2)) * CLOVER_ROWS * 16 >= (1ULL << 32))
    return fail(DDQ_ERR_ARG, "lattice too large: the FP64 clover field of one parity (576 bytes a site, " +
                                 std::to_string(V / 2) + " sites) must stay below 4 GiB, i.e. V/2 <= 7456512");
  AllocScope scope;
  ddq_lattice* L = new ddq_lattice();
  for (int k = 0; k < 4; ++k) L->dims[k] = dims[k];
  L->anti = t_antiperiodic ? 1 : 0;
  L->V = V;
  L->Vh = V / 2;
  Geo& g = L->geo;
  for (int k = 0; k < 4; ++k) g.L[k] = dims[k];
  g.Lxh = dims[0] / 2;
  g.Vh = (int)L->Vh;
  g.sY = g.Lxh;
  g.sZ = g.Lxh * dims[1];
  g.sT = g.Lxh * dims[1] * dims[2];
  g.antiperiodic = L->anti;
  L->stream = (hipStream_t)hip_stream;
  {
    const int r0 = scratch_address(&L->device, &L->noalloc_ws);
    if (r0 != DDQ_OK) {
      delete L;
      return r0;
    }
  }
  long long nb = (L->nvec() + 255) / 256;
  L->nbx = (int)(nb > 1024 ? 1024 : nb);
  int r = L->partial.ensure((size_t)L->nbx * 256 * sizeof(d2_t));
  if (r == DDQ_OK) r = L->small.ensure(4096 * sizeof(double));
  if (r == DDQ_OK) r = ensure_host(L, 4096 * sizeof(double));
  if (r != DDQ_OK) {
    ddq_destroy_lattice(L);
    return r;
  }
  *out = L;
  return DDQ_OK;
}

int ddq_destroy_lattice(ddq_lattice* L) {
  if (!L) return DDQ_OK;
  dfree(L->U);
  for (int p = 0; p < 4; ++p) {
    for (int q = 0; q < 2; ++q) {
      dfree(L->links[p][q]);
      dfree(L->clov[p][q]);
    }
    L->tmp[p].release();
  }
  dfree(L->clov_oo);
  L->scratch64.release();
  L->scratch32.release();
  L->oe_ws64.release();
  L->oe_ws32.release();
  for (int q = 0; q < 2; ++q) {
    L->sap_links[q].release();
    L->sap_clov[q].release();
    L->sap_rlinks[q].release();
    L->sap_rclov[q].release();
  }
  L->force_ws.release();
  L->partial.release();
  L->small.release();
  if (L->host) (void)hipHostFree(L->host);
  for (hipEvent_t e : L->ev) (void)hipEventDestroy(e);
  delete L;
  return DDQ_OK;
}

int ddq_set_stream(ddq_lattice* L, void* hip_stream) {
  CHK(check_lat(L));
  L->stream = (hipStream_t)hip_stream;
  return DDQ_OK;
}

int ddq_lattice_size(const ddq_lattice* L, int64_t* volume, int64_t* half_volume) {
  CHK(check_lat(L));
  if (volume) *volume = L->V;
  if (half_volume) *half_volume = L->Vh;
  return DDQ_OK;
}

int ddq_reserve(ddq_lattice* L, int max_nrhs, int max_m, unsigned what) {
  CHK(check_lat(L));
  if (max_nrhs < 1 || max_nrhs > 4096 || max_m < 0 || max_m > 128)
    return fail(DDQ_ERR_ARG, "max_nrhs must be in [1, 4096] and max_m in [0, 128]");
  if (what & ~(unsigned)(DDQ_RESERVE_SOLVE | DDQ_RESERVE_FULL | DDQ_RESERVE_SAP | DDQ_RESERVE_FORCE))
    return fail(DDQ_ERR_ARG, "unknown reservation flag");
  AllocScope scope;
  L->res_nrhs = std::max(L->res_nrhs, max_nrhs);
  L->res_m = std::max(L->res_m, max_m);
  L->res_what |= what;
  return reserve_impl(L);
}

int ddq_set_gauge(ddq_lattice* L, const void* U, int U_on_device, unsigned storage_flags) {
  CHK(check_lat(L));
  AllocScope scope;
  if (!U) return fail(DDQ_ERR_ARG, "U is null");
  if (storage_flags == 0) storage_flags = DDQ_STORE_F64 | DDQ_STORE_F32;
  if (storage_flags &
      ~(unsigned)(DDQ_STORE_F64 | DDQ_STORE_F32 | DDQ_STORE_F32_LINK12 | DDQ_STORE_F16 | DDQ_STORE_BF16))
    return fail(DDQ_ERR_ARG, "unknown storage flag");
  if (storage_flags & DDQ_STORE_F32_LINK12) storage_flags |= DDQ_STORE_F32;
  L->have_gauge = false;
  L->have_clover = false;
  L->sap_prec = -1;
  L->sap_res_ok = false;
  const size_t ubytes = (size_t)L->V * 4 * 9 * 16;
  if (!L->U) CHK(dalloc(&L->U, ubytes));
  HIPCHK(hipMemcpyAsync(L->U, U, ubytes, U_on_device ? hipMemcpyDeviceToDevice : hipMemcpyHostToDevice,
                        L->stream));
  const size_t n = (size_t)8 * 9 * field_vh((int)L->Vh);  // complex entries per parity
  for (int q = 0; q < 2; ++q)
    if (!L->links[DDQ_F64][q]) {
      CHK(dalloc(&L->links[DDQ_F64][q], n * 16));
      HIPCHK(hipMemsetAsync(L->links[DDQ_F64][q], 0, n * 16, L->stream));  // block padding
    }
  HIPCHK(launch_pack_gauge_f64(L->geo, (const d2_t*)L->U, (d2_t*)L->links[DDQ_F64][0],
                               (d2_t*)L->links[DDQ_F64][1], L->stream));
  L->link12 = (storage_flags & DDQ_STORE_F32_LINK12) != 0;
  if (storage_flags & DDQ_STORE_F32) {
    for (int q = 0; q < 2; ++q) {
      if (!L->links[DDQ_F32][q]) CHK(dalloc(&L->links[DDQ_F32][q], n * 8));
      if (L->link12)
        HIPCHK(launch_links_to_f32_12((const d2_t*)L->links[DDQ_F64][q], L->links[DDQ_F32][q], (int)L->Vh,
                                      L->stream));
      else
        HIPCHK(launch_field_to_f32((const d2_t*)L->links[DDQ_F64][q], L->links[DDQ_F32][q], 4, LINK_ROWS,
                                   (int)L->Vh, L->stream));
    }
  } else {
    for (int q = 0; q < 2; ++q) dfree(L->links[DDQ_F32][q]);
    L->h16_clover32 = false;  // no FP32 clover blocks without FP32 storage
  }
  // 16-bit storage: 12-real links, 3 element rows per direction
  const size_t n16 = (size_t)4 * 3 * field_vh((int)L->Vh) * 16;
  for (int prec : {DDQ_F16, DDQ_BF16}) {
    const unsigned flag = prec == DDQ_F16 ? DDQ_STORE_F16 : DDQ_STORE_BF16;
    for (int q = 0; q < 2; ++q) {
      if (!(storage_flags & flag)) {
        dfree(L->links[prec][q]);
        dfree(L->clov[prec][q]);
        continue;
      }
      if (!L->links[prec][q]) {
        CHK(dalloc(&L->links[prec][q], n16));
        HIPCHK(hipMemsetAsync(L->links[prec][q], 0, n16, L->stream));  // block padding
      }
      HIPCHK(launch_links_to_h16(h16_kind(prec), (const d2_t*)L->links[DDQ_F64][q], L->links[prec][q], (int)L->Vh,
                                 L->stream));
    }
  }
  L->store = storage_flags | DDQ_STORE_F64;
  CHK(reserve_impl(L));
  L->have_gauge = true;
  return DDQ_OK;
}

int ddq_set_clover(ddq_lattice* L, double c_sw, double m0) {
  CHK(check_lat(L));
  AllocScope scope;
  if (!L->have_gauge) return fail(DDQ_ERR_STATE, "ddq_set_gauge has not been called");
  if (!std::isfinite(c_sw) || !std::isfinite(m0)) return fail(DDQ_ERR_ARG, "c_sw and m0 must be finite");
  L->have_clover = false;
  L->sap_prec = -1;
  L->sap_res_ok = false;
  const size_t n = (size_t)36 * field_vh((int)L->Vh);  // (re, im) slots per parity
  for (int q = 0; q < 2; ++q)
    if (!L->clov[DDQ_F64][q]) {
      CHK(dalloc(&L->clov[DDQ_F64][q], n * 16));
      HIPCHK(hipMemsetAsync(L->clov[DDQ_F64][q], 0, n * 16, L->stream));  // block padding
    }
  if (!L->clov_oo) {
    CHK(dalloc(&L->clov_oo, n * 16));
    HIPCHK(hipMemsetAsync(L->clov_oo, 0, n * 16, L->stream));
  }
  int* flag = (int*)L->small.p;
  HIPCHK(hipMemsetAsync(flag, 0, sizeof(int), L->stream));
  HIPCHK(launch_clover_build(L->geo, (const d2_t*)L->U, c_sw, m0, (d2_t*)L->clov[DDQ_F64][0],
                             (d2_t*)L->clov[DDQ_F64][1], (d2_t*)L->clov_oo, flag, L->stream));
  CHK(fetch(L, flag, sizeof(int)));
  int notpd = ((int*)L->host)[0];
  if (notpd) return fail(DDQ_ERR_NOT_PD, "a 6x6 clover block is not positive definite");
  if (L->links[DDQ_F32][0]) {
    for (int q = 0; q < 2; ++q) {
      if (!L->clov[DDQ_F32][q]) CHK(dalloc(&L->clov[DDQ_F32][q], n * 8));
      HIPCHK(launch_field_to_f32((const d2_t*)L->clov[DDQ_F64][q], L->clov[DDQ_F32][q], 1, CLOVER_ROWS,
                                 (int)L->Vh, L->stream));
    }
  }
  const size_t n16 = (size_t)10 * field_vh((int)L->Vh) * 16;  // 16-bit: 10 element rows
  for (int prec : {DDQ_F16, DDQ_BF16}) {
    if (!L->links[prec][0]) continue;
    for (int q = 0; q < 2; ++q) {
      if (!L->clov[prec][q]) {
        CHK(dalloc(&L->clov[prec][q], n16));
        HIPCHK(hipMemsetAsync(L->clov[prec][q], 0, n16, L->stream));
      }
      HIPCHK(launch_clover_to_h16(h16_kind(prec), (const d2_t*)L->clov[DDQ_F64][q], L->clov[prec][q], (int)L->Vh,
                                  L->stream));
    }
  }
  HIPCHK(hipStreamSynchronize(L->stream));
  L->c_sw = c_sw;
  L->m0 = m0;
  L->have_clover = true;
  return DDQ_OK;
}

int ddq_get_clover(ddq_lattice* L, void* A_ee, void* A_oo_inv) {
  CHK(check_ready(L, DDQ_F64));
  if (A_ee) HIPCHK(launch_clover_export(L->geo, (const d2_t*)L->clov[DDQ_F64][0], (d2_t*)A_ee, L->stream));
  if (A_oo_inv)
    HIPCHK(launch_clover_export(L->geo, (const d2_t*)L->clov[DDQ_F64][1], (d2_t*)A_oo_inv, L->stream));
  HIPCHK(hipStreamSynchronize(L->stream));
  return DDQ_OK;
}

int ddq_pack_parity(ddq_lattice* L, int prec, int nrhs, int parity, const void* full, void* v) {
  CHK(check_lat(L));
  CHK(check_prec(prec));
  if (nrhs < 1 || (parity != 0 && parity != 1) || !full || !v) return fail(DDQ_ERR_ARG, "bad pack arguments");
  if (prec == DDQ_F64)
    HIPCHK(launch_pack_parity<double>(L->geo, parity, nrhs, (const d2_t*)full, (d2_t*)v, L->stream));
  else
    HIPCHK(launch_pack_parity<float>(L->geo, parity, nrhs, (const f2_t*)full, (f2_t*)v, L->stream));
  return DDQ_OK;
}

int ddq_unpack_parity(ddq_lattice* L, int prec, int nrhs, int parity, const void* v, void* full) {
  CHK(check_lat(L));
  CHK(check_prec(prec));
  if (nrhs < 1 || (parity != 0 && parity != 1) || !full || !v) return fail(DDQ_ERR_ARG, "bad unpack arguments");
  if (prec == DDQ_F64)
    HIPCHK(launch_unpack_parity<double>(L->geo, parity, nrhs, (const d2_t*)v, (d2_t*)full, L->stream));
  else
    HIPCHK(launch_unpack_parity<float>(L->geo, parity, nrhs, (const f2_t*)v, (f2_t*)full, L->stream));
  return DDQ_OK;
}

int ddq_apply_schur(ddq_lattice* L, int prec, int nrhs, const void* x_e, void* y_e, int dagger) {
  CHK(check_ready(L, prec));
  if (nrhs < 1 || !x_e || !y_e) return fail(DDQ_ERR_ARG, "bad apply arguments");
  if (x_e == y_e) return fail(DDQ_ERR_ARG, "x_e and y_e must not overlap");
  CHK(ensure_tmp(L, prec, nrhs));
  if (is16(prec)) {
    if (dagger) return fail(DDQ_ERR_ARG, "the 16-bit path has no daggered apply");
    return schur16(L, prec, nrhs, x_e, y_e);
  }
  if (prec == DDQ_F64) return schur<double>(L, prec, nrhs, (const d2_t*)x_e, (d2_t*)y_e, dagger != 0);
  return schur<float>(L, prec, nrhs, (const f2_t*)x_e, (f2_t*)y_e, dagger != 0);
}

int ddq_apply_schur_noalloc(ddq_lattice* L, int prec, int nrhs, const void* x_e, void* y_e, int dagger) {
  CHK(check_ready(L, prec));
  if (nrhs < 1 || !x_e || !y_e) return fail(DDQ_ERR_ARG, "bad apply arguments");
  if (x_e == y_e) return fail(DDQ_ERR_ARG, "x_e and y_e must not overlap");
  const size_t need = (size_t)nrhs * (size_t)L->nvec() * elem_bytes(prec);
  if (need > NOALLOC_SCRATCH_BYTES)
    return fail(DDQ_ERR_ARG, "ddq_apply_schur_noalloc: u_o needs " + std::to_string(need) +
                                 " bytes, more than the fixed work space of " + std::to_string(NOALLOC_SCRATCH_BYTES) +
                                 " bytes (nrhs x V/2 x 12 x " + std::to_string(elem_bytes(prec)) + " bytes)");
  int dev = -1;
  HIPCHK(hipGetDevice(&dev));
  if (dev != L->device || !L->noalloc_ws)
    return fail(DDQ_ERR_STATE, "ddq_apply_schur_noalloc: the lattice was created on device " +
                                   std::to_string(L->device) + ", the current device is " + std::to_string(dev));
  struct Guard {
    Guard() { g_no_alloc_call = true; }
    ~Guard() { g_no_alloc_call = false; }
  } guard;
  void* u = L->noalloc_ws;
  if (is16(prec)) {
    if (dagger) return fail(DDQ_ERR_ARG, "the 16-bit path has no daggered apply");
    return schur16(L, prec, nrhs, x_e, y_e, u);
  }
  if (prec == DDQ_F64) return schur<double>(L, prec, nrhs, (const d2_t*)x_e, (d2_t*)y_e, dagger != 0, (d2_t*)u);
  return schur<float>(L, prec, nrhs, (const f2_t*)x_e, (f2_t*)y_e, dagger != 0, (f2_t*)u);
}

int ddq_richardson_smooth(ddq_lattice* L, int prec, int nrhs, void* x_e, const void* b_e, int nsweeps,
                          double omega) {
  CHK(check_ready(L, prec));
  if (nrhs < 1 || !x_e || !b_e || nsweeps < 0) return fail(DDQ_ERR_ARG, "bad smoother arguments");
  if (x_e == b_e) return fail(DDQ_ERR_ARG, "x_e and b_e must not overlap");
  CHK(ensure_tmp(L, prec, nrhs));
  if (is16(prec)) return sweeps16(L, prec, nrhs, x_e, b_e, nsweeps, (float)omega);
  if (prec == DDQ_F64) return sweeps<double>(L, prec, nrhs, (d2_t*)x_e, (const d2_t*)b_e, nsweeps, omega);
  return sweeps<float>(L, prec, nrhs, (f2_t*)x_e, (const f2_t*)b_e, nsweeps, (float)omega);
}

namespace {
int check_mrhs(ddq_lattice* L, int nrhs) {
  CHK(check_ready(L, DDQ_F32));
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS)
    return fail(DDQ_ERR_ARG, "nrhs must be in [1, " + std::to_string(MRHS_MAX_NRHS) + "]");
  if ((uint64_t)L->Vh * 96u * (uint64_t)nrhs >= (1ULL << 32))
    return fail(DDQ_ERR_ARG, "an mrhs vector (V/2 x 96 x nrhs bytes) must stay below 4 GiB");
  return DDQ_OK;
}
int check_engine(int engine) {
  if (engine != DDQ_ENGINE_VALU && engine != DDQ_ENGINE_MFMA)
    return fail(DDQ_ERR_ARG, "engine must be DDQ_ENGINE_VALU or DDQ_ENGINE_MFMA");
  return DDQ_OK;
}
}  // namespace

int ddq_set_sweep_chunks(ddq_lattice* L, int nc) {
  CHK(check_lat(L));
  if (nc < 0 || nc > L->dims[3]) return fail(DDQ_ERR_ARG, "nc must be in [0, Lt]");
  L->sweep_chunks = nc;
  return DDQ_OK;
}

int ddq_set_h16_clover(ddq_lattice* L, int fp32) {
  CHK(check_lat(L));
  if (fp32 != 0 && fp32 != 1) return fail(DDQ_ERR_ARG, "fp32 must be 0 or 1");
  if (fp32 && !L->links[DDQ_F32][0]) return fail(DDQ_ERR_STATE, "FP32 clover blocks need DDQ_STORE_F32");
  L->h16_clover32 = fp32 != 0;
  return DDQ_OK;
}

int ddq_mrhs_pack(ddq_lattice* L, int nrhs, const void* src, void* dst) {
  CHK(check_lat(L));
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS || !src || !dst) return fail(DDQ_ERR_ARG, "bad mrhs pack arguments");
  if (src == dst) return fail(DDQ_ERR_ARG, "src and dst must not overlap");
  HIPCHK(launch_mrhs_layout(src, dst, nrhs, (int)L->Vh, true, L->stream));
  return DDQ_OK;
}

int ddq_mrhs_unpack(ddq_lattice* L, int nrhs, const void* src, void* dst) {
  CHK(check_lat(L));
  if (nrhs < 1 || nrhs > MRHS_MAX_NRHS || !src || !dst) return fail(DDQ_ERR_ARG, "bad mrhs unpack arguments");
  if (src == dst) return fail(DDQ_ERR_ARG, "src and dst must not overlap");
  HIPCHK(launch_mrhs_layout(src, dst, nrhs, (int)L->Vh, false, L->stream));
  return DDQ_OK;
}

int ddq_mrhs_set_launch(ddq_lattice* L, int order, int lds_kb, int tsteps, int stage) {
  CHK(check_lat(L));
  if (order != MRHS_ORDER_PLAIN && order != MRHS_ORDER_SLAB && order != MRHS_ORDER_TWALK)
    return fail(DDQ_ERR_ARG, "order must be 0, 1 or 2");
  if (lds_kb < 0 || lds_kb > 160) return fail(DDQ_ERR_ARG, "lds_kb must be in [0, 160]");
  if (order == MRHS_ORDER_TWALK && (tsteps < 1 || tsteps > L->dims[3] / 2))
    return fail(DDQ_ERR_ARG, "tsteps must be in [1, Lt / 2] for the t walk");
  if (stage != 0 && stage != 1) return fail(DDQ_ERR_ARG, "stage must be 0 or 1");
  L->mrhs_stage = stage;
  L->mrhs_order = order;
  L->mrhs_lds_kb = lds_kb;
  L->mrhs_tsteps = order == MRHS_ORDER_TWALK ? tsteps : 0;
  return DDQ_OK;
}

// kernels A and B of the mrhs stencil on t-chunks in the order of sweep_chunked when
// ddq_set_sweep_chunks asked for them (the default here is one range: at 24^3 x 48 with 12
// right-hand sides, ranges measured slower — their launches are too small for the chip),
// never with the t walk
static int mrhs_pass(ddq_lattice* L, int nrhs, int engine, const void* x, const void* b, void* u, void* out,
                     float omega, int mode) {
  int nc = L->sweep_chunks > 0 ? L->sweep_chunks : 1;
  nc = std::max(1, std::min(nc, L->dims[3]));
  if (L->mrhs_order == MRHS_ORDER_TWALK) nc = 1;
  if (nc == 1) {
    HIPCHK(run_mrhs(L, nrhs, M_HOP_CLINV, engine, x, nullptr, nullptr, u, 0.f));
    HIPCHK(run_mrhs(L, nrhs, mode, engine, u, x, b, out, omega));
    return DDQ_OK;
  }
  const int lt = L->dims[3];
  auto lo = [&](int c) { return (int)((long long)c * lt / nc); };
  auto A = [&](int c) { return run_mrhs(L, nrhs, M_HOP_CLINV, engine, x, nullptr, nullptr, u, 0.f, lo(c), lo(c + 1) - lo(c)); };
  auto B = [&](int c) { return run_mrhs(L, nrhs, mode, engine, u, x, b, out, omega, lo(c), lo(c + 1) - lo(c)); };
  HIPCHK(A(nc - 1));
  HIPCHK(A(0));
  for (int c = 0; c + 1 < nc; ++c) {
    if (c + 1 < nc - 1) HIPCHK(A(c + 1));
    HIPCHK(B(c));
  }
  HIPCHK(B(nc - 1));
  return DDQ_OK;
}

int ddq_mrhs_apply_schur(ddq_lattice* L, int nrhs, const void* x_e, void* y_e, int engine) {
  CHK(check_mrhs(L, nrhs));
  CHK(check_engine(engine));
  if (!x_e || !y_e) return fail(DDQ_ERR_ARG, "bad apply arguments");
  if (x_e == y_e) return fail(DDQ_ERR_ARG, "x_e and y_e must not overlap");
  CHK(ensure_tmp(L, DDQ_F32, nrhs));
  return mrhs_pass(L, nrhs, engine, x_e, nullptr, L->tmp[DDQ_F32].p, y_e, 0.f, M_APPLY);
}

int ddq_mrhs_richardson_smooth(ddq_lattice* L, int nrhs, void* x_e, const void* b_e, int nsweeps, double omega,
                               int engine) {
  CHK(check_mrhs(L, nrhs));
  CHK(check_engine(engine));
  if (!x_e || !b_e || nsweeps < 0) return fail(DDQ_ERR_ARG, "bad smoother arguments");
  if (x_e == b_e) return fail(DDQ_ERR_ARG, "x_e and b_e must not overlap");
  CHK(ensure_tmp(L, DDQ_F32, nrhs));
  void* u = L->tmp[DDQ_F32].p;
  for (int k = 0; k < nsweeps; ++k) CHK(mrhs_pass(L, nrhs, engine, x_e, b_e, u, x_e, (float)omega, M_RICH));
  return DDQ_OK;
}

int ddq_set_multi_rhs_tile(ddq_lattice* L, int nrhs, const ddq_mr_tile* tile) {
  CHK(check_lat(L));
  if (!tile || nrhs < 2) return fail(DDQ_ERR_ARG, "need a tile and nrhs >= 2");
  MrTile t;
  t.nb = tile->nb;
  t.g = tile->waves;
  t.xmap = tile->xcd_map;
  t.passes = tile->passes < 1 ? 1 : tile->passes;
  t.lds_kb = tile->lds_kb;
  if ((t.nb != 0 && !hop_rb_supported(M_RICH, false, nrhs, t)) || t.xmap < XMAP_SLAB || t.xmap > 1024 ||
      (t.nb == 0 && (t.passes != 1 || t.lds_kb != 0)))
    return fail(DDQ_ERR_ARG, "tile: nb must be 0 or divide nrhs / passes with nb <= 4, waves 1 or 4, xcd_map "
                             "-1..1024, passes dividing nrhs, lds_kb 0..160 (passes 1, lds_kb 0 for nb = 0)");
  for (auto& e : L->tiles)
    if (e.first == nrhs) {
      e.second = t;
      return DDQ_OK;
    }
  L->tiles.push_back({nrhs, t});
  return DDQ_OK;
}

int ddq_tune_multi_rhs(ddq_lattice* L, int nrhs, int reps, ddq_mr_tile* results, int max_results, int* n_results,
                       ddq_mr_tile* chosen) {
  CHK(check_ready(L, DDQ_F32));
  AllocScope scope;  // a set-up call: its two work vectors are its own
  if (nrhs < 2 || nrhs > 4096) return fail(DDQ_ERR_ARG, "nrhs must be in [2, 4096]");
  if (reps < 1) reps = 5;
  const size_t N = (size_t)nrhs * L->nvec();
  CHK(L->scratch32.ensure(2 * N * 8));
  CHK(ensure_tmp(L, DDQ_F32, nrhs));
  f2_t* x = (f2_t*)L->scratch32.p;
  f2_t* b = x + N;
  HIPCHK(hipMemsetAsync(x, 0, 2 * N * 8, L->stream));
  std::vector<ddq_mr_tile> cand;
  for (int xm : {XMAP_SLAB, 0})  // one right-hand side per thread, the 64-site x 4 mapping
    cand.push_back({0, 4, xm, 0.0, 1, 0});
  for (int nb = 1; nb <= MR_MAX_NB; ++nb)
    if (nrhs % nb == 0)
      for (int g : {1, 4})
        for (int xm : {XMAP_SLAB, 0, 1, 8, 32}) cand.push_back({nb, g, xm, 0.0, 1, 0});
  // fewer right-hand sides or fewer workgroups in flight: slab order, RHS passes and an
  // LDS cap on the resident workgroups
  for (int nb = 1; nb <= MR_MAX_NB; ++nb)
    for (int passes : {1, 2, 3, 4})
      if (nrhs % passes == 0 && (nrhs / passes) % nb == 0 && nrhs / passes >= 2)
        for (int g : {1, 4})
          for (int lds : {0, 48, 64, 96})
            if (passes > 1 || lds > 0) cand.push_back({nb, g, XMAP_SLAB, 0.0, passes, lds});
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIPCHK(hipEventCreate(&e0));
  hipError_t he = hipEventCreate(&e1);
  if (he != hipSuccess) {
    (void)hipEventDestroy(e0);
    HIPCHK(he);
  }
  const bool prof = L->prof_on;
  L->prof_on = false;
  int rc = DDQ_OK;
  size_t best = 0;
  for (size_t k = 0; k < cand.size() && rc == DDQ_OK; ++k) {
    rc = ddq_set_multi_rhs_tile(L, nrhs, &cand[k]);
    if (rc == DDQ_OK) rc = sweeps<float>(L, DDQ_F32, nrhs, x, b, 1, 0.1f);  // warm-up
    if (rc == DDQ_OK && hipEventRecord(e0, L->stream) != hipSuccess) rc = fail(DDQ_ERR_HIP, "event record");
    if (rc == DDQ_OK) rc = sweeps<float>(L, DDQ_F32, nrhs, x, b, reps, 0.1f);
    if (rc == DDQ_OK && hipEventRecord(e1, L->stream) != hipSuccess) rc = fail(DDQ_ERR_HIP, "event record");
    float ms = 0.f;
    if (rc == DDQ_OK && (hipEventSynchronize(e1) != hipSuccess || hipEventElapsedTime(&ms, e0, e1) != hipSuccess))
      rc = fail(DDQ_ERR_HIP, "event timing");
    cand[k].ms = ms / reps;
    if (rc == DDQ_OK && cand[k].ms < cand[best].ms) best = k;
  }
  L->prof_on = prof;
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (rc != DDQ_OK) {
    for (auto it = L->tiles.begin(); it != L->tiles.end(); ++it)
      if (it->first == nrhs) {
        L->tiles.erase(it);
        break;
      }
    return rc;
  }
  CHK(ddq_set_multi_rhs_tile(L, nrhs, &cand[best]));
  bool have = false;
  for (auto& m : L->tile_ms)
    if (m.first == nrhs) {
      m.second = cand[best].ms;
      have = true;
    }
  if (!have) L->tile_ms.push_back({nrhs, cand[best].ms});
  if (results)
    for (int k = 0; k < max_results && k < (int)cand.size(); ++k) results[k] = cand[k];
  if (n_results) *n_results = (int)cand.size();
  if (chosen) *chosen = cand[best];
  return DDQ_OK;
}

// ddq_autotune: the cache file holds one JSON object per line inside a "tiles" array, so
// a line-wise reader suffices; lines it does not recognise are dropped on rewrite.
namespace {
struct TileEntry {
  std::string key;
  int nrhs = 0;
  ddq_mr_tile t{};
};

bool parse_tile_line(const std::string& line, TileEntry& e) {
  const std::string k0 = "\"key\": \"";
  const size_t a = line.find(k0);
  if (a == std::string::npos) return false;
  const size_t b = line.find('"', a + k0.size());
  if (b == std::string::npos) return false;
  e.key = line.substr(a + k0.size(), b - a - k0.size());
  e.t.passes = 1;
  e.t.lds_kb = 0;
  if (std::sscanf(line.c_str() + b + 1,
                  ", \"nrhs\": %d, \"nb\": %d, \"waves\": %d, \"xcd_map\": %d, \"passes\": %d, \"lds_kb\": %d, \"ms\": %lf",
                  &e.nrhs, &e.t.nb, &e.t.waves, &e.t.xcd_map, &e.t.passes, &e.t.lds_kb, &e.t.ms) == 7)
    return true;
  return std::sscanf(line.c_str() + b + 1, ", \"nrhs\": %d, \"nb\": %d, \"waves\": %d, \"xcd_map\": %d, \"ms\": %lf",
                     &e.nrhs, &e.t.nb, &e.t.waves, &e.t.xcd_map, &e.t.ms) == 5;
}
}  // namespace

int ddq_autotune(ddq_lattice* L, const char* cache_json_path) {
  CHK(check_lat(L));
  if (!cache_json_path || !*cache_json_path) return fail(DDQ_ERR_ARG, "cache_json_path is null or empty");
  // a tile is valid for one device kind, lattice extent and FP32 link storage
  int dev = 0;
  HIPCHK(hipGetDevice(&dev));
  hipDeviceProp_t prop;
  HIPCHK(hipGetDeviceProperties(&prop, dev));
  char key[256];
  std::snprintf(key, sizeof key, "%s/%dcu/%dx%dx%dx%d/%s", prop.gcnArchName, prop.multiProcessorCount, L->dims[0],
                L->dims[1], L->dims[2], L->dims[3], L->link12 ? "link12" : "link18");
  std::vector<TileEntry> cache;
  if (FILE* f = std::fopen(cache_json_path, "r")) {
    char buf[1024];
    while (std::fgets(buf, sizeof buf, f)) {
      TileEntry e;
      if (parse_tile_line(buf, e)) cache.push_back(e);
    }
    std::fclose(f);
  }
  // cached tiles of this key fill the counts the lattice has no tile for
  for (const TileEntry& e : cache)
    if (e.key == key && !L->tile_for(e.nrhs)) {
      if (ddq_set_multi_rhs_tile(L, e.nrhs, &e.t) != DDQ_OK)
        return fail(DDQ_ERR_ARG, std::string("invalid cached tile in ") + cache_json_path + " for " + key);
      L->tile_ms.push_back({e.nrhs, e.t.ms});
    }
  // the lattice's tiles replace the cache's entries of this key
  std::vector<TileEntry> out;
  for (const TileEntry& e : cache)
    if (e.key != key) out.push_back(e);
  for (const auto& t : L->tiles) {
    TileEntry e;
    e.key = key;
    e.nrhs = t.first;
    e.t = {t.second.nb, t.second.g, t.second.xmap, 0.0, t.second.passes, t.second.lds_kb};
    for (const auto& m : L->tile_ms)
      if (m.first == t.first) e.t.ms = m.second;
    out.push_back(e);
  }
  const std::string tmp = std::string(cache_json_path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return fail(DDQ_ERR_ARG, std::string("cannot write ") + tmp);
  std::fprintf(f, "{\"ddq_autotune\": 1, \"tiles\": [\n");
  for (size_t k = 0; k < out.size(); ++k)
    std::fprintf(f,
                 " {\"key\": \"%s\", \"nrhs\": %d, \"nb\": %d, \"waves\": %d, \"xcd_map\": %d, \"passes\": %d, "
                 "\"lds_kb\": %d, \"ms\": %.6g}%s\n",
                 out[k].key.c_str(), out[k].nrhs, out[k].t.nb, out[k].t.waves, out[k].t.xcd_map, out[k].t.passes,
                 out[k].t.lds_kb, out[k].t.ms, k + 1 < out.size() ? "," : "");
  std::fprintf(f, "]}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), cache_json_path) != 0)
    return fail(DDQ_ERR_ARG, std::string("cannot write ") + cache_json_path);
  return DDQ_OK;
}

int ddq_estimate_lambda_max(ddq_lattice* L, int iters, const void* v0, double* out) {
  CHK(check_ready(L, DDQ_F64));
  if (iters < 1 || !v0 || !out) return fail(DDQ_ERR_ARG, "bad power-iteration arguments");
  if (iters > 4000) return fail(DDQ_ERR_ARG, "at most 4000 power iterations");
  CHK(ensure_tmp(L, DDQ_F64, 1));
  const long long n = L->nvec();
  CHK(L->scratch64.ensure(2 * (size_t)n * 16));
  d2_t* v = (d2_t*)L->scratch64.p;
  d2_t* w = v + n;
  double* nrm = (double*)L->small.p;  // nrm[0] = |v0|^2, nrm[1 + k] = |D_S v_k|^2
  CHK(norm2_dev(L, (const d2_t*)v0, n, nrm));
  HIPCHK(launch_scale_dev(v, (const d2_t*)v0, nrm, n, L->stream));
  for (int k = 0; k < iters; ++k) {
    CHK(schur<double>(L, DDQ_F64, 1, v, w, false));
    CHK(norm2_dev(L, w, n, nrm + 1 + k));
    HIPCHK(launch_scale_dev(v, w, nrm + 1 + k, n, L->stream));
  }
  CHK(fetch(L, nrm, (size_t)(iters + 1) * sizeof(double)));
  double lg = 0.0;
  for (int k = 0; k < iters; ++k) lg += 0.5 * std::log(L->host[1 + k]);
  if (!(L->host[0] > 0.0)) return fail(DDQ_ERR_ARG, "v0 is zero");
  if (!std::isfinite(lg)) return fail(DDQ_ERR_NONFINITE, "power iteration produced a non-finite norm");
  *out = std::exp(lg / iters);
  return DDQ_OK;
}

int ddq_oe_prepare(ddq_lattice* L, int nrhs, const void* b, void* bt_e) {
  CHK(check_ready(L, DDQ_F64));
  if (nrhs < 1 || !b || !bt_e) return fail(DDQ_ERR_ARG, "bad prepare arguments");
  if (b == bt_e) return fail(DDQ_ERR_ARG, "b and bt_e must not overlap");
  CHK(L->scratch64.ensure((size_t)nrhs * L->nvec() * 16));
  return prepare_impl(L, nrhs, (const d2_t*)b, (d2_t*)bt_e, (d2_t*)L->scratch64.p);
}

int ddq_oe_reconstruct(ddq_lattice* L, int nrhs, const void* x_e, const void* b, void* x) {
  CHK(check_ready(L, DDQ_F64));
  if (nrhs < 1 || !x_e || !b || !x) return fail(DDQ_ERR_ARG, "bad reconstruct arguments");
  if (x == b || x == x_e) return fail(DDQ_ERR_ARG, "x must not overlap b or x_e");
  const size_t nb = (size_t)nrhs * L->nvec();
  CHK(L->scratch64.ensure(2 * nb * 16));
  d2_t* bo = (d2_t*)L->scratch64.p;
  return reconstruct_impl(L, nrhs, (const d2_t*)x_e, (const d2_t*)b, (d2_t*)x, bo, bo + nb);
}

int ddq_convert_parity(ddq_lattice* L, int nrhs, int src_prec, const void* src, int dst_prec, void* dst) {
  CHK(check_lat(L));
  CHK(check_prec(src_prec));
  CHK(check_prec(dst_prec));
  if (nrhs < 1 || !src || !dst) return fail(DDQ_ERR_ARG, "bad conversion arguments");
  if (src_prec == dst_prec) {
    HIPCHK(hipMemcpyAsync(dst, src, (size_t)nrhs * L->nvec() * elem_bytes(src_prec), hipMemcpyDeviceToDevice,
                          L->stream));
  } else if (src_prec == DDQ_F64 && dst_prec == DDQ_F32) {
    HIPCHK(launch_parity_to_f32(dst, (const d2_t*)src, nrhs, (int)L->Vh, L->stream));
  } else if (src_prec == DDQ_F32 && dst_prec == DDQ_F64) {
    HIPCHK(launch_parity_to_f64((d2_t*)dst, src, nrhs, (int)L->Vh, L->stream));
  } else if (src_prec == DDQ_F64 && is16(dst_prec)) {
    HIPCHK(launch_parity_to_h16(h16_kind(dst_prec), dst, (const d2_t*)src, 1.0, nrhs, (int)L->Vh, L->stream));
  } else if (is16(src_prec) && dst_prec == DDQ_F64) {
    HIPCHK(launch_parity_from_h16(h16_kind(src_prec), (d2_t*)dst, src, 1.0, nrhs, (int)L->Vh, L->stream));
  } else if (is16(src_prec) && dst_prec == DDQ_F32) {
    HIPCHK(launch_h16_to_f32(h16_kind(src_prec), dst, src, 1.0f, nrhs, (int)L->Vh, L->stream));
  } else {
    return fail(DDQ_ERR_ARG, "unsupported conversion (narrow to 16 bits from FP64)");
  }
  return DDQ_OK;
}

int ddq_backward_apply(ddq_lattice* L, int prec, int nrhs, const void* grad_y_e, void* grad_x_e) {
  return ddq_apply_schur(L, prec, nrhs, grad_y_e, grad_x_e, 1);
}

int ddq_backward_link_force(ddq_lattice* L, const void* chi_e, const void* phi_e, void* G, void* F,
                            int accumulate) {
  CHK(check_ready(L, DDQ_F64));
  if (!chi_e || !phi_e) return fail(DDQ_ERR_ARG, "chi_e and phi_e must be non-null");
  if (!G && !F) return DDQ_OK;
  const long long n = L->nvec();
  const size_t need = (size_t)(2 * n + L->V * 54) * 16;
  CHK(L->force_ws.ensure(need));
  CHK(ensure_tmp(L, DDQ_F64, 1));
  d2_t* psi = (d2_t*)L->force_ws.p;
  d2_t* lam = psi + n;
  d2_t* W = lam + n;
  // psi_o = A_oo^-1 H_oe phi_e ;  lambda_o = A_oo^-1 (H^H)_oe chi_e  (kernel A, plain and dagger)
  HIPCHK(kernel_A<double>(L, DDQ_F64, 1, (const d2_t*)phi_e, psi, false));
  HIPCHK(kernel_A<double>(L, DDQ_F64, 1, (const d2_t*)chi_e, lam, true));
  HIPCHK(launch_force(L->geo, (const d2_t*)L->U, (const d2_t*)chi_e, lam, (const d2_t*)phi_e, psi, L->c_sw, W,
                      (d2_t*)G, (double*)F, accumulate, L->stream));
  return DDQ_OK;
}

int ddq_stream_copy(void* dst, const void* src, int64_t bytes, int nontemporal, void* hip_stream) {
  if (!dst || !src || bytes < 0 || (bytes & 15) || (((uintptr_t)dst | (uintptr_t)src) & 15))
    return fail(DDQ_ERR_ARG, "stream copy needs 16-byte aligned pointers and a multiple of 16 bytes");
  if (bytes == 0) return DDQ_OK;
  HIPCHK(launch_stream_copy(dst, src, bytes, nontemporal != 0, (hipStream_t)hip_stream));
  return DDQ_OK;
}

int ddq_stencil_stream(ddq_lattice* L, int prec, int kernel, const void* in, const void* x, const void* b, void* out) {
  CHK(check_ready(L, prec));
  if (prec != DDQ_F32 && prec != DDQ_F64) return fail(DDQ_ERR_ARG, "the stencil stream probe takes DDQ_F32 or DDQ_F64");
  if (kernel < 0 || kernel > 2) return fail(DDQ_ERR_ARG, "kernel must be 0 (A), 1 (B apply) or 2 (B Richardson)");
  if (!in || !out || (kernel >= 1 && !x) || (kernel == 2 && !b)) return fail(DDQ_ERR_ARG, "missing vector");
  const int mode = kernel == 0 ? M_HOP_CLINV : (kernel == 1 ? M_APPLY : M_RICH);
  const int p_out = kernel == 0 ? 1 : 0;
  auto run = [&](auto tag) -> hipError_t {
    using T = decltype(tag);
    HopArgs<T> a = hop_args<T>(L, prec, p_out);
    a.in = (const pair<T>*)in;
    a.x = (const pair<T>*)x;
    a.b = (const pair<T>*)b;
    a.out = (pair<T>*)out;
    a.nrhs = 1;
    std::string name = std::string("stream_") + mode_name(mode) +
                       (prec == DDQ_F64 ? "_f64" : (a.link12 ? "_f32l12" : "_f32"));
    return prof_launch(L, name, hop_bytes(L, prec, mode, 1), [&]() { return launch_hop_stream<T>(a, mode, L->stream); });
  };
  if (prec == DDQ_F64)
    HIPCHK(run(double{}));
  else
    HIPCHK(run(float{}));
  return DDQ_OK;
}

bool ranges_overlap(const void* a, size_t na, const void* b, size_t nb) {
  const uintptr_t pa = (uintptr_t)a, pb = (uintptr_t)b;
  return pa < pb + nb && pb < pa + na;
}

int coarse_storage(int storage) {
  return storage == DDQ_F32 ? COARSE_F32 : storage == DDQ_F16 ? COARSE_F16 : storage == DDQ_BF16 ? COARSE_BF16 : -1;
}

int check_coarse(const int cdims[4], int nv, int storage, long long* packed_bytes) {
  if (coarse_storage(storage) < 0)
    return fail(DDQ_ERR_ARG, "coarse blocks are stored as DDQ_F32, DDQ_F16 or DDQ_BF16");
  const long long n = coarse_packed_bytes(cdims, nv, coarse_storage(storage));
  if (n < 0) return fail(DDQ_ERR_ARG, "coarse extents must be >= 1 with at most 2^25 sites, and 1 <= N_v <= 32");
  if (packed_bytes) *packed_bytes = n;
  return DDQ_OK;
}

int ddq_coarse_packed_bytes(const int cdims[4], int nv, int storage, int64_t* bytes) {
  if (!cdims || !bytes) return fail(DDQ_ERR_ARG, "null argument");
  long long n = 0;
  CHK(check_coarse(cdims, nv, storage, &n));
  *bytes = n;
  return DDQ_OK;
}

int ddq_coarse_pack_blocks(const int cdims[4], int nv, int storage, int prec, const void* blocks, void* packed,
                           void* hip_stream) {
  if (!cdims || !blocks || !packed) return fail(DDQ_ERR_ARG, "null argument");
  if (prec != DDQ_F64 && prec != DDQ_F32) return fail(DDQ_ERR_ARG, "blocks are complex128 (DDQ_F64) or complex64 (DDQ_F32)");
  if (((uintptr_t)packed & 15) || ((uintptr_t)blocks & (prec == DDQ_F64 ? 15 : 7)))
    return fail(DDQ_ERR_ARG, "misaligned blocks or packed array");
  long long packed_bytes = 0;
  CHK(check_coarse(cdims, nv, storage, &packed_bytes));
  const size_t sites = (size_t)cdims[0] * cdims[1] * cdims[2] * cdims[3];
  if (ranges_overlap(blocks, sites * 9 * 4 * nv * nv * (prec == DDQ_F64 ? 16 : 8), packed, (size_t)packed_bytes))
    return fail(DDQ_ERR_ARG, "packed must not overlap blocks");
  HIPCHK(launch_coarse_pack(cdims, nv, coarse_storage(storage), prec == DDQ_F64, blocks, packed,
                            (hipStream_t)hip_stream));
  return DDQ_OK;
}

int ddq_coarse_apply(const int cdims[4], int nv, int storage, int nrhs, const void* packed, const void* v, void* y,
                     int rhs_tiles_per_wave, int product, void* hip_stream) {
  if (!cdims || !packed || !v || !y) return fail(DDQ_ERR_ARG, "null argument");
  CHK(check_coarse(cdims, nv, storage, nullptr));
  if (nrhs < 1 || nrhs > 65535 * 16) return fail(DDQ_ERR_ARG, "nrhs must be in 1 .. 1048560");
  if (rhs_tiles_per_wave < 0 || rhs_tiles_per_wave > 4) return fail(DDQ_ERR_ARG, "rhs_tiles_per_wave must be 0 .. 4");
  if (product < 0 || product > 2) return fail(DDQ_ERR_ARG, "product must be 0 (default), 1 (four) or 2 (three real products)");
  if (((uintptr_t)packed & 15) || (((uintptr_t)v | (uintptr_t)y) & 7)) return fail(DDQ_ERR_ARG, "misaligned argument");
  const size_t vbytes = (size_t)cdims[0] * cdims[1] * cdims[2] * cdims[3] * 2 * nv * nrhs * 8;
  if (ranges_overlap(v, vbytes, y, vbytes)) return fail(DDQ_ERR_ARG, "y must not overlap v");
  HIPCHK(launch_coarse_apply(cdims, nv, coarse_storage(storage), nrhs, rhs_tiles_per_wave, product, packed, v, y,
                             (hipStream_t)hip_stream));
  return DDQ_OK;
}

int ddq_profile_begin(ddq_lattice* L) {
  CHK(check_lat(L));
  L->prof_on = true;
  L->ev_used = 0;
  L->kind_name.clear();
  L->kind_ms.clear();
  L->kind_n.clear();
  L->kind_bytes.clear();
  return DDQ_OK;
}

int ddq_profile_end(ddq_lattice* L, ddq_kernel_stats* out, int max_entries, int* n_out) {
  CHK(check_lat(L));
  if (!L->prof_on) return fail(DDQ_ERR_STATE, "ddq_profile_begin has not been called");
  CHK(prof_flush(L));
  L->prof_on = false;
  const int n = (int)L->kind_name.size();
  if (n_out) *n_out = n;
  for (int k = 0; k < n && k < max_entries && out; ++k) {
    std::memset(out[k].name, 0, sizeof(out[k].name));
    std::strncpy(out[k].name, L->kind_name[k].c_str(), sizeof(out[k].name) - 1);
    out[k].launches = L->kind_n[k];
    out[k].total_ms = L->kind_ms[k];
    out[k].bytes_per_launch = L->kind_n[k] > 0 ? L->kind_bytes[k] / L->kind_n[k] : 0.0;
  }
  return DDQ_OK;
}

}  // extern "C"

// ===========================================================================
// GMRES(m) of Alg. 2 on D_S, flexible and mixed precision
// ===========================================================================
namespace {

struct Givens {
  double c;
  cd s;
};

// rotate (a, b) -> (r, 0) with G = [[c, s], [-conj(s), c]], c real
Givens make_givens(cd a, cd b) {
  double na = std::abs(a), nb = std::abs(b);
  if (nb == 0.0) return {1.0, 0.0};
  if (na == 0.0) return {0.0, std::conj(b) / nb};
  double rho = std::hypot(na, nb);
  return {na / rho, (a / na) * std::conj(b) / rho};
}

// Restarted GMRES(m) of Alg. 2 on device vectors of n complex128 numbers, flexible
// when Z is given (z_k = M v_k kept, x += Z y): resid(x, r) forms r = b - A x in FP64,
// precop(v, z, w) forms z = M v (z = v when Z is null) and w = A z.  Classical
// Gram-Schmidt in `passes` passes, Givens rotations on the host, a cycle ends at
// max(target, red * beta) or on breakdown; convergence only on the recomputed
// residual at a restart.  x is updated in place; V holds m + 1 vectors, Z m, w one.
struct KrylovOps {
  std::function<int(const d2_t*, d2_t*)> resid;
  std::function<int(const d2_t*, d2_t*, d2_t*)> precop;
};
struct KrylovRun {
  int cycles = 0, iters = 0;
  double beta = 0.0;
};

int gmres_core(ddq_lattice* L, long long n, d2_t* x, d2_t* V, d2_t* Z, d2_t* w, int m, int max_cycles,
               double target, double red, int passes, const KrylovOps& ops, KrylovRun& run, int& status) {
  const bool flexible = Z != nullptr;
  d2_t* hdev = (d2_t*)L->small.p;        // [0, 128): first pass, [128, 256): second pass
  double* ndev = (double*)(hdev + 256);  // |w|^2
  CHK(ensure_host(L, 4096 * sizeof(double)));
  std::vector<cd> Hcol(m + 2), g(m + 2), y(m + 1);
  std::vector<std::vector<cd>> R(m, std::vector<cd>(m + 1));
  std::vector<Givens> rot(m);
  status = DDQ_NOT_CONVERGED;
  double beta = 0.0;
  int cycles, iters = 0;
  for (cycles = 0;; ++cycles) {
    // r = b - A x (FP64), the iterative-refinement residual
    CHK(ops.resid(x, V));
    CHK(norm_host(L, V, n, &beta));
    if (!std::isfinite(beta)) return fail(DDQ_ERR_NONFINITE, "residual norm is not finite");
    if (beta <= target) {
      status = DDQ_OK;
      break;
    }
    if (cycles == max_cycles) break;
    HIPCHK(launch_scale(V, V, 1.0 / beta, n, L->stream));
    std::fill(g.begin(), g.end(), cd(0.0));
    g[0] = beta;
    const double cycle_target = std::max(target, red * beta);
    int k_used = 0;
    for (int k = 0; k < m; ++k) {
      d2_t* vk = V + (size_t)k * n;
      d2_t* zk = flexible ? Z + (size_t)k * n : vk;
      CHK(ops.precop(vk, zk, w));
      // classical Gram-Schmidt: h = V^H w, w -= V h (twice for CGS2)
      const int kk = k + 1;
      for (int pass = 0; pass < passes; ++pass) {
        d2_t* h = hdev + pass * 128;
        HIPCHK(launch_dot_partial(V, n, kk, w, n, (d2_t*)L->partial.p, L->nbx, L->stream));
        HIPCHK(launch_reduce_partial((const d2_t*)L->partial.p, L->nbx, kk, h, L->stream));
        HIPCHK(launch_update(w, V, n, kk, h, -1.0, n, L->stream));
      }
      CHK(norm2_dev(L, w, n, ndev));
      CHK(fetch(L, hdev, 256 * sizeof(d2_t) + sizeof(double)));
      const double* hh = L->host;
      for (int j = 0; j < kk; ++j)
        Hcol[j] = passes == 2 ? cd(hh[2 * j] + hh[256 + 2 * j], hh[2 * j + 1] + hh[256 + 2 * j + 1])
                              : cd(hh[2 * j], hh[2 * j + 1]);
      const double hn = std::sqrt(hh[512]);
      if (!std::isfinite(hn)) return fail(DDQ_ERR_NONFINITE, "Arnoldi norm is not finite");
      Hcol[kk] = hn;
      // apply the previous rotations, then a new one
      for (int j = 0; j < k; ++j) {
        cd t = rot[j].c * Hcol[j] + rot[j].s * Hcol[j + 1];
        Hcol[j + 1] = -std::conj(rot[j].s) * Hcol[j] + rot[j].c * Hcol[j + 1];
        Hcol[j] = t;
      }
      rot[k] = make_givens(Hcol[k], Hcol[kk]);
      Hcol[k] = rot[k].c * Hcol[k] + rot[k].s * Hcol[kk];
      Hcol[kk] = 0.0;
      g[kk] = -std::conj(rot[k].s) * g[k];
      g[k] = rot[k].c * g[k];
      for (int j = 0; j <= k; ++j) R[k][j] = Hcol[j];
      ++iters;
      k_used = kk;
      const double est = std::abs(g[kk]);
      if (est <= cycle_target || hn <= 1e-14 * beta) break;
      HIPCHK(launch_scale(V + (size_t)kk * n, w, 1.0 / hn, n, L->stream));
    }
    // y = R^-1 g, x += Z y (or V y)
    for (int j = k_used - 1; j >= 0; --j) {
      cd sum = g[j];
      for (int q = j + 1; q < k_used; ++q) sum -= R[q][j] * y[q];
      y[j] = sum / R[j][j];
    }
    double* yh = L->host;
    for (int j = 0; j < k_used; ++j) {
      yh[2 * j] = y[j].real();
      yh[2 * j + 1] = y[j].imag();
    }
    d2_t* ydev = hdev;
    HIPCHK(hipMemcpyAsync(ydev, yh, (size_t)k_used * sizeof(d2_t), hipMemcpyHostToDevice, L->stream));
    HIPCHK(launch_update(x, flexible ? Z : V, n, k_used, ydev, 1.0, n, L->stream));
    HIPCHK(hipStreamSynchronize(L->stream));  // yh is reused next cycle
  }
  run.cycles = cycles;
  run.iters = iters;
  run.beta = beta;
  return DDQ_OK;
}

// Richardson preconditioner z = p_{R,nu}(D_S) v (Alg. 4, nu sweeps from zero) on nrhs
// FP64 parity vectors, with the sweeps in FP64 or in FP32 storage (b32, x32: FP32 work
// vectors; on return x32 holds z in FP32).  nu = 0 gives z = 0.
int rich_prec_impl(ddq_lattice* L, int nrhs, const d2_t* v, d2_t* z, int nu, double omega, int prec, f2_t* b32,
                   f2_t* x32) {
  const long long n = (long long)nrhs * L->nvec();
  if (nu == 0) {
    HIPCHK(hipMemsetAsync(z, 0, (size_t)n * 16, L->stream));
    if (prec == DDQ_F32) HIPCHK(hipMemsetAsync(x32, 0, (size_t)n * 8, L->stream));
    return DDQ_OK;
  }
  if (prec == DDQ_F64) {
    HIPCHK(launch_scale(z, v, omega, n, L->stream));  // the first sweep from zero
    return sweeps<double>(L, DDQ_F64, nrhs, z, v, nu - 1, omega);
  }
  HIPCHK(launch_parity_to_f32(b32, v, nrhs, (int)L->Vh, L->stream));
  HIPCHK(launch_scale_f32(x32, b32, (float)omega, n, L->stream));
  CHK(sweeps<float>(L, DDQ_F32, nrhs, x32, b32, nu - 1, (float)omega));
  HIPCHK(launch_parity_to_f64(z, x32, nrhs, (int)L->Vh, L->stream));
  return DDQ_OK;
}

// y = D x for nrhs full FP64 vectors (eq. 1): y_e = A_ee x_e - H_eo x_o and
// y_o = A_oo x_o - H_oe x_e, kernel B's APPLY mode on each parity (the odd one with
// the undivided A_oo).  ws: 4 nrhs parity vectors.
int dirac_impl(ddq_lattice* L, int nrhs, const d2_t* x, d2_t* y, d2_t* ws) {
  const size_t nb = (size_t)nrhs * L->nvec();
  d2_t *xe = ws, *xo = ws + nb, *ye = ws + 2 * nb, *yo = ws + 3 * nb;
  HIPCHK(launch_pack_parity<double>(L->geo, 0, nrhs, x, xe, L->stream));
  HIPCHK(launch_pack_parity<double>(L->geo, 1, nrhs, x, xo, L->stream));
  HIPCHK(kernel_B<double>(L, DDQ_F64, nrhs, M_APPLY, xo, xe, nullptr, ye, 0.0, false));
  HopArgs<double> a = hop_args<double>(L, DDQ_F64, 1);
  a.clov = (const d2_t*)L->clov_oo;
  a.in = xe;
  a.x = xo;
  a.out = yo;
  HIPCHK(run_hop<double>(L, a, M_APPLY, false, nrhs));
  HIPCHK(launch_unpack_parity<double>(L->geo, 0, nrhs, ye, y, L->stream));
  HIPCHK(launch_unpack_parity<double>(L->geo, 1, nrhs, yo, y, L->stream));
  return DDQ_OK;
}

// z = M_nu r for nrhs full FP64 vectors (Sect. 2.4.5): eq. 2 with D_S^-1 replaced by
// p_{R,nu}(D_S) -- prepare, nu Richardson sweeps from zero in `prec`, reconstruct.
// ws: 4 nrhs FP64 parity vectors; b32, x32: nrhs FP32 parity vectors (prec DDQ_F32).
int smoother_impl(ddq_lattice* L, int nrhs, const d2_t* r, d2_t* z, int nu, double omega, int prec, d2_t* ws,
                  f2_t* b32, f2_t* x32) {
  const size_t nb = (size_t)nrhs * L->nvec();
  d2_t *bt = ws, *xe = ws + nb, *bo = ws + 2 * nb, *xo = ws + 3 * nb;
  CHK(prepare_impl(L, nrhs, r, bt, bo));
  CHK(rich_prec_impl(L, nrhs, bt, xe, nu, omega, prec, b32, x32));
  return reconstruct_impl(L, nrhs, xe, r, z, bo, xo);
}

// the smoother's and the full operator's work vectors (8 FP64 + 2 FP32 parity vectors
// per right-hand side)
int oe_workspace(ddq_lattice* L, int nrhs, int prec, d2_t** ws64, f2_t** ws32) {
  const size_t nb = (size_t)nrhs * L->nvec();
  CHK(L->oe_ws64.ensure(8 * nb * 16));
  *ws64 = (d2_t*)L->oe_ws64.p;
  *ws32 = nullptr;
  if (prec == DDQ_F32) {
    CHK(L->oe_ws32.ensure(2 * nb * 8));
    CHK(ensure_tmp(L, DDQ_F32, nrhs));
    *ws32 = (f2_t*)L->oe_ws32.p;
  }
  return ensure_tmp(L, DDQ_F64, nrhs);
}

}  // namespace

namespace {

// |b - D x| of one full FP64 system from its parity halves x_e, x_o (eq. 1 on the two
// parities, kernel B's residual mode: r_e = b_e - A_ee x_e + H_eo x_o and r_o = b_o -
// A_oo x_o + H_oe x_e); t_e, t_o: work parity vectors
int full_residual_norm(ddq_lattice* L, const d2_t* xe, const d2_t* xo, const d2_t* b, d2_t* t_e, d2_t* t_o,
                       double* out) {
  const long long n = L->nvec();
  HIPCHK(launch_pack_parity<double>(L->geo, 0, 1, b, t_e, L->stream));
  HIPCHK(kernel_B<double>(L, DDQ_F64, 1, M_RESID, xo, xe, t_e, t_e, 0.0, false));
  HIPCHK(launch_pack_parity<double>(L->geo, 1, 1, b, t_o, L->stream));
  HopArgs<double> a = hop_args<double>(L, DDQ_F64, 1);
  a.clov = (const d2_t*)L->clov_oo;
  a.in = xe;
  a.x = xo;
  a.b = t_o;
  a.out = t_o;
  HIPCHK(run_hop<double>(L, a, M_RESID, false, 1));
  double* d = (double*)L->small.p;
  CHK(norm2_dev(L, t_e, n, d));
  CHK(norm2_dev(L, t_o, n, d + 1));
  CHK(fetch(L, d, 2 * sizeof(double)));
  *out = std::sqrt(L->host[0] + L->host[1]);
  return DDQ_OK;
}

int oe_solve_one(ddq_lattice* L, void* x, const void* b, const ddq_gmres_params* P, ddq_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = P->m;
  if (m < 1 || m > 128) return fail(DDQ_ERR_ARG, "cycle length m must be in [1, 128]");
  if (!(L->res_what & DDQ_RESERVE_SOLVE) || m > L->res_m)
    return fail(DDQ_ERR_STATE, "the solver's work space is reserved for m <= " + std::to_string(L->res_m) +
                                   " (ddq_reserve with DDQ_RESERVE_SOLVE and max_m >= " + std::to_string(m) + ")");
  if (P->max_cycles < 0 || !(P->tol >= 0.0) || P->smoother_sweeps < 0)
    return fail(DDQ_ERR_ARG, "bad max_cycles, tol or smoother_sweeps");
  if (P->inner_prec != DDQ_F64 && P->inner_prec != DDQ_F32)
    return fail(DDQ_ERR_ARG, "inner_prec must be DDQ_F64 or DDQ_F32");
  const bool lo = P->inner_prec == DDQ_F32;
  if (lo) CHK(check_ready(L, DDQ_F32));
  const int sp = P->smoother_prec;  // 16-bit storage for the Richardson preconditioner
  const bool s16 = is16(sp) && P->smoother_sweeps > 0;
  if (s16) {
    if (!lo) return fail(DDQ_ERR_ARG, "a 16-bit smoother needs inner_prec = DDQ_F32");
    CHK(check_ready(L, sp));
  }
  const int nu = P->smoother_sweeps;
  const bool flexible = nu > 0 || lo;
  if (P->orth_passes < 0 || P->orth_passes > 2) return fail(DDQ_ERR_ARG, "orth_passes must be 0, 1 or 2");
  const int passes = P->orth_passes == 1 ? 1 : 2;
  const double red = P->inner_reduction > 0.0 ? P->inner_reduction : (lo ? 1e-5 : 0.0);
  const long long n = L->nvec();
  const size_t vb = (size_t)n * 16;

  // FP64 work: bt, xe, w, V[0..m], Z[0..m-1]
  const size_t nv64 = 3 + (size_t)(m + 1) + (flexible ? (size_t)m : 0);
  CHK(L->scratch64.ensure(nv64 * vb));
  CHK(ensure_tmp(L, DDQ_F64, 1));
  d2_t* base = (d2_t*)L->scratch64.p;
  d2_t* bt = base;
  d2_t* xe = base + n;
  d2_t* w = base + 2 * n;
  d2_t* V = base + 3 * n;
  d2_t* Z = flexible ? V + (size_t)(m + 1) * n : nullptr;
  // FP32 work: b32, x32, w32
  f2_t *b32 = nullptr, *x32 = nullptr, *w32 = nullptr;
  if (lo) {
    CHK(L->scratch32.ensure(3 * (size_t)n * 8));
    CHK(ensure_tmp(L, DDQ_F32, 1));
    if (s16) CHK(ensure_tmp(L, sp, 1));
    b32 = (f2_t*)L->scratch32.p;
    x32 = b32 + n;
    w32 = b32 + 2 * n;
  }

  int applies64 = 0, applies_lo = 0;
  // |b| of the full right-hand side (2 parities: 2n complex numbers)
  double bnorm;
  CHK(norm_host(L, (const d2_t*)b, 2 * n, &bnorm));
  if (!std::isfinite(bnorm)) return fail(DDQ_ERR_NONFINITE, "right-hand side is not finite");
  const double target = P->tol * bnorm;

  // eq. 2: b~_e, initial x_e from the even half of x
  CHK(prepare_impl(L, 1, (const d2_t*)b, bt, w));
  HIPCHK(launch_pack_parity<double>(L->geo, 0, 1, (const d2_t*)x, xe, L->stream));

  KrylovOps ops;
  ops.resid = [&](const d2_t* xx, d2_t* r) -> int {
    ++applies64;
    return resid<double>(L, DDQ_F64, 1, xx, bt, r);
  };
  // z_k = M v_k, w = D_S z_k
  ops.precop = [&](const d2_t* vk, d2_t* zk, d2_t* ww) -> int {
    if (lo) {
      if (s16) {
        // the same sweeps on 16-bit storage: v_k (unit norm) scaled by sqrt(n) so its
        // entries are of order one, b16 = s v, x16 = omega s v, then back with 1/s
        // (the sweeps are linear in b, so the scale cancels exactly)
        const double sc = std::sqrt((double)n);
        void* b16 = b32;
        void* x16 = (char*)b32 + (size_t)n * 4;
        HIPCHK(launch_parity_to_h16(h16_kind(sp), b16, vk, sc, 1, (int)L->Vh, L->stream));
        HIPCHK(launch_parity_to_h16(h16_kind(sp), x16, vk, sc * P->omega, 1, (int)L->Vh, L->stream));
        CHK(sweeps16(L, sp, 1, x16, b16, nu - 1, (float)P->omega));
        HIPCHK(launch_h16_to_f32(h16_kind(sp), x32, x16, (float)(1.0 / sc), 1, (int)L->Vh, L->stream));
        applies_lo += nu - 1;
      } else if (nu > 0) {
        CHK(rich_prec_impl(L, 1, vk, zk, nu, P->omega, DDQ_F32, b32, x32));
        applies_lo += nu - 1;
      } else {
        HIPCHK(launch_parity_to_f32(x32, vk, 1, (int)L->Vh, L->stream));
      }
      if (s16 || nu == 0) HIPCHK(launch_parity_to_f64(zk, x32, 1, (int)L->Vh, L->stream));
      CHK(schur<float>(L, DDQ_F32, 1, x32, w32, false));
      ++applies_lo;
      HIPCHK(launch_parity_to_f64(ww, w32, 1, (int)L->Vh, L->stream));
    } else {
      if (nu > 0) {
        CHK(rich_prec_impl(L, 1, vk, zk, nu, P->omega, DDQ_F64, nullptr, nullptr));
        applies64 += nu - 1;
      }
      CHK(schur<double>(L, DDQ_F64, 1, zk, ww, false));
      ++applies64;
    }
    return DDQ_OK;
  };
  // GMRES on D_S to |b~_e - D_S x_e| <= schur_target, then eq. 2's reconstruction and the
  // full residual |b - D x| in FP64.  The two agree in exact arithmetic; when rounding
  // leaves the full residual above tol |b|, the Schur target is lowered by the observed
  // ratio and the restarts continue, so a converged status always means the full bar.
  double schur_target = target, full = 0.0;
  int status = DDQ_NOT_CONVERGED, cycles = 0, iters = 0;
  for (;;) {
    KrylovRun run;
    CHK(gmres_core(L, n, xe, V, Z, w, m, P->max_cycles - cycles, schur_target, red, passes, ops, run, status));
    cycles += run.cycles;
    iters += run.iters;
    CHK(reconstruct_impl(L, 1, xe, (const d2_t*)b, (d2_t*)x, V, w));  // x_o in w
    CHK(full_residual_norm(L, xe, w, (const d2_t*)b, V, V + n, &full));
    if (!std::isfinite(full)) return fail(DDQ_ERR_NONFINITE, "full residual norm is not finite");
    if (full <= target) {
      status = DDQ_OK;
      break;
    }
    status = DDQ_NOT_CONVERGED;
    if (cycles >= P->max_cycles || run.beta <= 0.0) break;
    schur_target = std::min(0.5 * schur_target, 0.9 * run.beta * target / full);
  }
  if (info) {
    info->cycles = cycles;
    info->iters = iters;
    info->applies_f64 = applies64;
    info->applies_lo = applies_lo;
    info->true_relres = bnorm > 0 ? full / bnorm : 0.0;
    info->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status == DDQ_NOT_CONVERGED) g_err = "GMRES stopped at max_cycles";
  return status;
}

}  // namespace

extern "C" int ddq_oe_gmres_solve(ddq_lattice* L, int nrhs, void* x, const void* b, const ddq_gmres_params* P,
                                  ddq_solve_info* info) {
  CHK(check_ready(L, DDQ_F64));
  if (nrhs < 1 || !x || !b || !P) return fail(DDQ_ERR_ARG, "nrhs >= 1; x, b and params must be non-null");
  const size_t full = 2 * (size_t)L->nvec() * 16;  // bytes of one full FP64 vector
  if (ranges_overlap(x, nrhs * full, b, nrhs * full)) return fail(DDQ_ERR_ARG, "x and b must not overlap");
  int worst = DDQ_OK;
  for (int r = 0; r < nrhs; ++r) {
    const int st = oe_solve_one(L, (char*)x + r * full, (const char*)b + r * full, P, info ? info + r : nullptr);
    if (st < 0) return st;
    if (st == DDQ_NOT_CONVERGED) worst = st;
  }
  if (worst == DDQ_NOT_CONVERGED) g_err = "GMRES stopped at max_cycles for at least one right-hand side";
  return worst;
}

extern "C" int ddq_apply_dirac(ddq_lattice* L, int nrhs, const void* x, void* y) {
  CHK(check_ready(L, DDQ_F64));
  if (nrhs < 1 || !x || !y) return fail(DDQ_ERR_ARG, "bad apply arguments");
  if (x == y) return fail(DDQ_ERR_ARG, "x and y must not overlap");
  d2_t* ws64;
  f2_t* ws32;
  CHK(oe_workspace(L, nrhs, DDQ_F64, &ws64, &ws32));
  return dirac_impl(L, nrhs, (const d2_t*)x, (d2_t*)y, ws64);
}

extern "C" int ddq_oe_smoother(ddq_lattice* L, int nrhs, const void* r, void* z, int nsweeps, double omega,
                               int prec) {
  CHK(check_ready(L, DDQ_F64));
  if (prec != DDQ_F64 && prec != DDQ_F32) return fail(DDQ_ERR_ARG, "prec must be DDQ_F64 or DDQ_F32");
  if (prec == DDQ_F32) CHK(check_ready(L, DDQ_F32));
  if (nrhs < 1 || !r || !z || nsweeps < 0 || !std::isfinite(omega))
    return fail(DDQ_ERR_ARG, "bad smoother arguments");
  if (r == z) return fail(DDQ_ERR_ARG, "r and z must not overlap");
  d2_t* ws64;
  f2_t* ws32;
  CHK(oe_workspace(L, nrhs, prec, &ws64, &ws32));
  const size_t nb = (size_t)nrhs * L->nvec();
  return smoother_impl(L, nrhs, (const d2_t*)r, (d2_t*)z, nsweeps, omega, prec, ws64 + 4 * nb, ws32,
                       ws32 ? ws32 + nb : nullptr);
}

namespace {

// SAP(n, m) of Alg. 1 on D x = b (full FP64 vectors), x updated in place: every sweep
// recomputes r = b - D x (FP64) on the blocks of a colour before that colour's block
// solves, which run in prec (DDQ_F64 or DDQ_F32).  x_zero: x is zero on entry, so the
// first colour's residual is b itself and is read from b.  ws64: the workspace of
// oe_workspace (r uses its upper half).
int sap_impl(ddq_lattice* L, int prec, d2_t* x, const d2_t* b, int n, int m, d2_t* ws64, bool x_zero = false) {
  d2_t* r = ws64 + 4 * (size_t)L->nvec();
  const bool f32 = prec == DDQ_F32;
  const bool l12 = f32 && L->link12;
  const size_t fvh = (size_t)field_vh((int)L->Vh);
  if (L->sap_prec != prec) {  // links and clover in SAP order, built once per gauge field and clover
    const int cpe = f32 ? 2 : 1;
    const int lrows = (l12 ? LINK12_ROWS : LINK_ROWS) / cpe, crows = CLOVER_ROWS / cpe;
    for (int q = 0; q < 2; ++q) {
      CHK(L->sap_links[q].ensure(4 * (size_t)lrows * fvh * 16));
      CHK(L->sap_clov[q].ensure((size_t)crows * fvh * 16));
      for (int mu = 0; mu < 4; ++mu)
        HIPCHK(launch_sap_reorder(L->geo, q, (const char*)L->links[prec][q] + (size_t)mu * lrows * fvh * 16,
                                  (char*)L->sap_links[q].p + (size_t)mu * lrows * fvh * 16, lrows, L->stream));
      HIPCHK(launch_sap_reorder(L->geo, q, L->clov[prec][q], L->sap_clov[q].p, crows, L->stream));
    }
    L->sap_prec = prec;
  }
  if (!L->sap_res_ok) {  // the residual's FP64 links and undivided clover blocks in SAP order
    for (int q = 0; q < 2; ++q) {
      CHK(L->sap_rlinks[q].ensure(4 * (size_t)LINK_ROWS * fvh * 16));
      CHK(L->sap_rclov[q].ensure((size_t)CLOVER_ROWS * fvh * 16));
      for (int mu = 0; mu < 4; ++mu)
        HIPCHK(launch_sap_reorder(L->geo, q,
                                  (const char*)L->links[DDQ_F64][q] + (size_t)mu * LINK_ROWS * fvh * 16,
                                  (char*)L->sap_rlinks[q].p + (size_t)mu * LINK_ROWS * fvh * 16, LINK_ROWS,
                                  L->stream));
    }
    HIPCHK(launch_sap_reorder(L->geo, 0, L->clov[DDQ_F64][0], L->sap_rclov[0].p, CLOVER_ROWS, L->stream));
    HIPCHK(launch_sap_reorder(L->geo, 1, L->clov_oo, L->sap_rclov[1].p, CLOVER_ROWS, L->stream));
    L->sap_res_ok = true;
  }
  // algorithmic bytes of one colour's launches, per site of that colour's blocks:
  // block solve -- the FP64 residual, the FP64 iterate (read and written), the links and
  // the clover blocks once; residual -- x (its own sites and, once, the other colour's),
  // b, r, the FP64 links and clover blocks.  On chip the block solves form r themselves:
  // the sum of both without r's store and load.
  const double per_site = 192 + 384 + (f32 ? (l12 ? 384 : 576) + 288 : 1152 + 576);
  const double per_site_res = 2 * 192 + 192 + 192 + 1152 + 576;
  const bool on_chip = sap_on_chip(L->geo, f32, l12);
  const std::string tag = "_mr" + std::to_string(m) + (f32 ? (l12 ? "_f32l12" : "_f32") : "_f64");
  const SapResidualSrc src{b, x, {L->sap_rlinks[0].p, L->sap_rlinks[1].p}, {L->sap_rclov[0].p, L->sap_rclov[1].p}};
  for (int it = 0; it < n; ++it)
    for (int colour = 0; colour < 2; ++colour) {
      const bool from_b = x_zero && it == 0 && colour == 0;  // r = b - D 0 = b
      if (!from_b && !on_chip)
        HIPCHK(prof_launch(L, "sap_residual_f64", (double)L->V / 2 * per_site_res, [&]() {
          return launch_sap_residual(L->geo, src, r, colour, L->stream);  // r = b - D x on the colour's blocks
        }));
      const bool fused = on_chip && !from_b;
      const double bytes = (double)L->V / 2 * (fused ? per_site + per_site_res - 2 * 192 : per_site);
      HIPCHK(prof_launch(L, (fused ? "sap_res_block" : "sap_block") + tag, bytes, [&]() {
        return launch_sap_blocks(L->geo, f32, l12, from_b ? b : r, x, L->sap_links[0].p, L->sap_links[1].p,
                                 L->sap_clov[0].p, L->sap_clov[1].p, colour, m, fused ? &src : nullptr,
                                 L->stream);
      }));
    }
  return DDQ_OK;
}

int check_sap(ddq_lattice* L, int n, int m) {
  if (n < 0 || m < 0) return fail(DDQ_ERR_ARG, "SAP sweeps and Minimal Residual steps must be >= 0");
  for (int mu = 0; mu < 4; ++mu)
    if (L->dims[mu] % 4 != 0) return fail(DDQ_ERR_ARG, "SAP blocks are 4^4: every extent must be a multiple of 4");
  return DDQ_OK;
}

// FGMRES(m) of Alg. 2 on the full D with right preconditioner precop_z (z = M v)
int fgmres_full(ddq_lattice* L, void* x, const void* b, const ddq_gmres_params* P, ddq_solve_info* info,
                d2_t* ws64, const std::function<int(const d2_t*, d2_t*)>& prec, const int* applies_lo,
                const int* applies_prec64) {
  auto t0 = std::chrono::steady_clock::now();
  const int m = P->m;
  if (P->orth_passes < 0 || P->orth_passes > 2) return fail(DDQ_ERR_ARG, "orth_passes must be 0, 1 or 2");
  if (m > L->res_m)
    return fail(DDQ_ERR_STATE, "the FGMRES work space is reserved for m <= " + std::to_string(L->res_m) +
                                   " (ddq_reserve with max_m >= " + std::to_string(m) + ")");
  const int passes = P->orth_passes == 1 ? 1 : 2;
  const long long n = 2 * L->nvec();  // complex numbers of a full vector
  const size_t vb = (size_t)n * 16;
  // FP64 work: w, V[0..m], Z[0..m-1] (full vectors)
  CHK(L->scratch64.ensure((1 + (size_t)(m + 1) + (size_t)m) * vb));
  d2_t* w = (d2_t*)L->scratch64.p;
  d2_t* V = w + n;
  d2_t* Z = V + (size_t)(m + 1) * n;
  double bnorm;
  CHK(norm_host(L, (const d2_t*)b, n, &bnorm));
  if (!std::isfinite(bnorm)) return fail(DDQ_ERR_NONFINITE, "right-hand side is not finite");
  int applies64 = 0;
  const double red = P->inner_reduction > 0.0 ? P->inner_reduction : 0.0;
  KrylovOps ops;
  ops.resid = [&](const d2_t* xx, d2_t* r) -> int {  // r = b - D x
    CHK(dirac_impl(L, 1, xx, r, ws64));
    ++applies64;
    HIPCHK(launch_scale(r, r, -1.0, n, L->stream));
    HIPCHK(launch_axpy(r, 1.0, 0.0, (const d2_t*)b, n, L->stream));
    return DDQ_OK;
  };
  ops.precop = [&](const d2_t* vk, d2_t* zk, d2_t* ww) -> int {  // z = M v, w = D z
    CHK(prec(vk, zk));
    CHK(dirac_impl(L, 1, zk, ww, ws64));
    ++applies64;
    return DDQ_OK;
  };
  KrylovRun run;
  int status = DDQ_NOT_CONVERGED;
  CHK(gmres_core(L, n, (d2_t*)x, V, Z, w, m, P->max_cycles, P->tol * bnorm, red, passes, ops, run, status));
  HIPCHK(hipStreamSynchronize(L->stream));
  if (info) {
    info->cycles = run.cycles;
    info->iters = run.iters;
    info->applies_f64 = applies64 + (applies_prec64 ? *applies_prec64 : 0);
    info->applies_lo = applies_lo ? *applies_lo : 0;
    info->true_relres = bnorm > 0 ? run.beta / bnorm : 0.0;
    info->t_total_ms =
        std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  }
  if (status == DDQ_NOT_CONVERGED) g_err = "FGMRES stopped at max_cycles";
  return status;
}

int check_fgmres(ddq_lattice* L, void* x, const void* b, const ddq_gmres_params* P) {
  CHK(check_ready(L, DDQ_F64));
  if (!x || !b || !P) return fail(DDQ_ERR_ARG, "x, b and params must be non-null");
  if (x == b) return fail(DDQ_ERR_ARG, "x and b must not overlap");
  if (P->m < 1 || P->m > 128) return fail(DDQ_ERR_ARG, "cycle length m must be in [1, 128]");
  if (P->max_cycles < 0 || !(P->tol >= 0.0)) return fail(DDQ_ERR_ARG, "bad max_cycles or tol");
  return DDQ_OK;
}

}  // namespace

extern "C" int ddq_sap_smooth(ddq_lattice* L, int prec, void* x, const void* b, int n, int m) {
  CHK(check_ready(L, DDQ_F64));
  if (prec != DDQ_F64 && prec != DDQ_F32) return fail(DDQ_ERR_ARG, "prec must be DDQ_F64 or DDQ_F32");
  CHK(check_ready(L, prec));
  if (!x || !b) return fail(DDQ_ERR_ARG, "bad SAP arguments");
  if (x == b) return fail(DDQ_ERR_ARG, "x and b must not overlap");
  CHK(check_sap(L, n, m));
  d2_t* ws64;
  f2_t* ws32;
  CHK(oe_workspace(L, 1, DDQ_F64, &ws64, &ws32));
  CHK(sap_impl(L, prec, (d2_t*)x, (const d2_t*)b, n, m, ws64));
  HIPCHK(hipStreamSynchronize(L->stream));
  return DDQ_OK;
}

extern "C" int ddq_fgmres_sap_solve(ddq_lattice* L, void* x, const void* b, const ddq_gmres_params* P,
                                    int sap_n, int sap_m, ddq_solve_info* info) {
  CHK(check_fgmres(L, x, b, P));
  CHK(check_sap(L, sap_n, sap_m));
  const int prec = P->inner_prec;
  if (prec != DDQ_F64 && prec != DDQ_F32) return fail(DDQ_ERR_ARG, "inner_prec must be DDQ_F64 or DDQ_F32");
  CHK(check_ready(L, prec));
  d2_t* ws64;
  f2_t* ws32;
  CHK(oe_workspace(L, 1, DDQ_F64, &ws64, &ws32));
  const long long nf = 2 * L->nvec();
  auto sap_prec = [&](const d2_t* v, d2_t* z) -> int {  // z = SAP(n, m) on D z = v from zero
    HIPCHK(hipMemsetAsync(z, 0, (size_t)nf * 16, L->stream));
    return sap_impl(L, prec, z, v, sap_n, sap_m, ws64, true);
  };
  return fgmres_full(L, x, b, P, info, ws64, sap_prec, nullptr, nullptr);
}

extern "C" int ddq_fgmres_solve(ddq_lattice* L, void* x, const void* b, const ddq_gmres_params* P,
                                ddq_solve_info* info) {
  CHK(check_fgmres(L, x, b, P));
  if (P->smoother_sweeps < 0 || !std::isfinite(P->omega)) return fail(DDQ_ERR_ARG, "bad smoother_sweeps or omega");
  const int prec = P->inner_prec;
  if (prec != DDQ_F64 && prec != DDQ_F32) return fail(DDQ_ERR_ARG, "inner_prec must be DDQ_F64 or DDQ_F32");
  if (prec == DDQ_F32) CHK(check_ready(L, DDQ_F32));
  if (P->smoother_prec != 0 && P->smoother_prec != prec)
    return fail(DDQ_ERR_ARG, "the odd-even smoother runs its sweeps in inner_prec (smoother_prec must be 0)");
  d2_t* ws64;
  f2_t* ws32;
  CHK(oe_workspace(L, 1, prec, &ws64, &ws32));
  const size_t nb = L->nvec();
  int applies_lo = 0, applies64 = 0;  // Schur applies of the sweeps (the first is a scaling)
  auto smoother = [&](const d2_t* v, d2_t* z) -> int {  // z = M_nu v
    CHK(smoother_impl(L, 1, v, z, P->smoother_sweeps, P->omega, prec, ws64 + 4 * nb, ws32,
                      ws32 ? ws32 + nb : nullptr));
    (prec == DDQ_F32 ? applies_lo : applies64) += P->smoother_sweeps > 0 ? P->smoother_sweeps - 1 : 0;
    return DDQ_OK;
  };
  return fgmres_full(L, x, b, P, info, ws64, smoother, &applies_lo, &applies64);
}

// ===========================================================================
// Batched flexible GMRES: several lattices, several right-hand sides each.
// Every (lattice, right-hand side) system runs Alg. 2 with eq. 2 around it, all
// in lock-step.  The preconditioner and operator stage of Arnoldi step k (FP32
// Richardson sweeps z = M v_k and w = D_S z for every right-hand side of every
// lattice, through the multi-right-hand-side kernels) is one hipGraph per step
// index, captured once and replayed every cycle; the FP64 orthogonalisation is
// batched over right-hand sides; the host synchronises once per Arnoldi step
// for the whole batch.
// ===========================================================================
struct ddq_batch {
  struct Sys {
    ddq_lattice* L = nullptr;
    int nrhs = 0;
    long long n = 0;  // complex numbers of one parity vector
    int nbx = 0;
    Grow w64, w32, small, partial;
    d2_t *bt = nullptr, *xe = nullptr, *w = nullptr, *z = nullptr, *V = nullptr, *Z = nullptr;
    void *b32 = nullptr, *x32 = nullptr, *w32v = nullptr;
    d2_t *h1 = nullptr, *h2 = nullptr, *y = nullptr;
    double *hn = nullptr, *f = nullptr;
    // cycle mode: the coefficients of every step of a cycle, [step][rhs][...]
    Grow cyc;
    d2_t *ch1 = nullptr, *ch2 = nullptr;
    double *chn = nullptr, *cf = nullptr;
    double omega = 0.0;
  };
  std::vector<Sys> sys;
  hipStream_t user = nullptr;    // the caller's stream: inputs are ordered on it
  hipStream_t stream = nullptr;  // the batch's own stream (captured)
  hipEvent_t ev = nullptr;
  std::vector<hipGraphExec_t> step_graph;  // one per Arnoldi step index
  std::vector<uintptr_t> graph_key;        // what the captured graphs bake in
  int sprec = DDQ_F32;                     // storage of the Richardson preconditioner
  int passes = 2;                          // Gram-Schmidt passes per Arnoldi step
  int cycle = 0;                           // 1: one graph per restart cycle of m steps
  double* host = nullptr;                  // pinned
  size_t host_bytes = 0;
  int res_m = 0, res_cycle = 0;            // ddq_batch_reserve: largest m, cycle mode reserved
};

namespace {

constexpr int BLD = 128;  // leading dimension of the per-system coefficient arrays

void batch_release_graphs(ddq_batch* B) {
  for (hipGraphExec_t e : B->step_graph)
    if (e) (void)hipGraphExecDestroy(e);
  B->step_graph.clear();
  B->graph_key.clear();
}

int batch_host(ddq_batch* B, size_t bytes) {
  if (bytes <= B->host_bytes) return DDQ_OK;
  if (g_alloc_depth == 0) return fail(DDQ_ERR_STATE, "batch host buffer too small: call ddq_batch_reserve");
  if (B->host) (void)hipHostFree(B->host);
  B->host = nullptr;
  B->host_bytes = 0;
  HIPCHK(hipHostMalloc((void**)&B->host, bytes, hipHostMallocDefault));
  B->host_bytes = bytes;
  return DDQ_OK;
}

// device scalars of one system: h1, h2 (BLD complex per right-hand side), |w|^2
// (contiguous, fetched in one copy), then y (BLD complex) and the scale factors
size_t batch_d2h_bytes(int nrhs, int steps = 1) { return (size_t)steps * nrhs * (2 * BLD * 16 + 8); }
size_t batch_h2d_doubles(int nrhs) { return (size_t)nrhs * (2 * BLD + 1); }

int batch_workspace(ddq_batch::Sys& S, int m, bool cycle) {
  const size_t N = (size_t)S.nrhs * S.n;  // complex numbers of a batched vector
  CHK(S.w64.ensure((size_t)(2 * m + 5) * N * 16));
  d2_t* p = (d2_t*)S.w64.p;
  S.bt = p;
  S.xe = p + N;
  S.w = p + 2 * N;
  S.z = p + 3 * N;
  S.V = p + 4 * N;                  // m + 1 vectors
  S.Z = S.V + (size_t)(m + 1) * N;  // m vectors
  CHK(S.w32.ensure(3 * N * 8));
  S.b32 = S.w32.p;
  S.x32 = (char*)S.w32.p + N * 8;
  S.w32v = (char*)S.w32.p + 2 * N * 8;
  CHK(S.small.ensure(batch_d2h_bytes(S.nrhs) + batch_h2d_doubles(S.nrhs) * 8));
  S.h1 = (d2_t*)S.small.p;
  S.h2 = S.h1 + (size_t)S.nrhs * BLD;
  S.hn = (double*)(S.h2 + (size_t)S.nrhs * BLD);
  S.y = (d2_t*)(S.hn + S.nrhs);
  S.f = (double*)(S.y + (size_t)S.nrhs * BLD);
  CHK(S.partial.ensure((size_t)S.nbx * S.nrhs * BLD * 16));
  if (cycle) {
    const size_t mr = (size_t)m * S.nrhs;
    CHK(S.cyc.ensure(batch_d2h_bytes(S.nrhs, m) + mr * 8));
    S.ch1 = (d2_t*)S.cyc.p;
    S.ch2 = S.ch1 + mr * BLD;
    S.chn = (double*)(S.ch2 + mr * BLD);
    S.cf = S.chn + mr;
  }
  CHK(ensure_tmp(S.L, DDQ_F32, S.nrhs));
  CHK(ensure_tmp(S.L, DDQ_F64, S.nrhs));
  return DDQ_OK;
}

// pinned host doubles of a solve: per system its D2H then its H2D block
size_t batch_host_doubles(const ddq_batch* B, int m, bool cycle) {
  size_t n = 0;
  for (const auto& S : B->sys) n += batch_d2h_bytes(S.nrhs, cycle ? m : 1) / 8 + batch_h2d_doubles(S.nrhs);
  return n;
}

// Arnoldi step k for every system, the body of one graph:
//   v_k = w f (k >= 1; f = 1/|w| per right-hand side, 0 once it has stopped),
//   z_k = M v_k (nu FP32 Richardson sweeps from zero, the first one folded into
//   x = omega b), w = D_S z_k in FP32, both widened to FP64,
//   CGS2: h = V^H w, w -= V h (twice), then |w|^2
int batch_step(ddq_batch* B, int k, int nu) {
  for (auto& S : B->sys) {
    ddq_lattice* L = S.L;
    const size_t N = (size_t)S.nrhs * S.n;
    d2_t* vk = S.V + (size_t)k * N;
    d2_t* zk = S.Z + (size_t)k * N;
    const int vh = (int)L->Vh;
    // per-step coefficient slots in cycle mode, else one set reused every step
    const size_t cs = (size_t)k * S.nrhs;
    d2_t* h1 = B->cycle ? S.ch1 + cs * BLD : S.h1;
    d2_t* h2 = B->cycle ? S.ch2 + cs * BLD : S.h2;
    double* hn = B->cycle ? S.chn + cs : S.hn;
    const double* fk = B->cycle ? S.cf + cs - S.nrhs : S.f;  // factor of v_k from step k - 1
    if (k > 0) HIPCHK(launch_scale_b(vk, S.w, fk, S.n, S.nrhs, B->stream));
    if (nu > 0 && is16(B->sprec)) {
      // 16-bit storage: scaled so that the unit-norm v_k has entries of order one
      const double sc = std::sqrt((double)S.n);
      void* b16 = S.b32;
      void* x16 = (char*)S.b32 + N * 4;
      HIPCHK(launch_parity_to_h16(h16_kind(B->sprec), b16, vk, sc, S.nrhs, vh, B->stream));
      HIPCHK(launch_parity_to_h16(h16_kind(B->sprec), x16, vk, sc * S.omega, S.nrhs, vh, B->stream));
      CHK(sweeps16(L, B->sprec, S.nrhs, x16, b16, nu - 1, (float)S.omega));
      HIPCHK(launch_h16_to_f32(h16_kind(B->sprec), S.x32, x16, (float)(1.0 / sc), S.nrhs, vh, B->stream));
    } else if (nu > 0) {
      HIPCHK(launch_parity_to_f32(S.b32, vk, S.nrhs, vh, B->stream));
      HIPCHK(launch_scale_f32((f2_t*)S.x32, (const f2_t*)S.b32, (float)S.omega, (long long)N, B->stream));
      CHK(sweeps<float>(L, DDQ_F32, S.nrhs, (f2_t*)S.x32, (const f2_t*)S.b32, nu - 1, (float)S.omega));
    } else {
      HIPCHK(launch_parity_to_f32(S.x32, vk, S.nrhs, vh, B->stream));
    }
    HIPCHK(launch_parity_to_f64(zk, S.x32, S.nrhs, vh, B->stream));
    CHK(schur<float>(L, DDQ_F32, S.nrhs, (const f2_t*)S.x32, (f2_t*)S.w32v, false));
    HIPCHK(launch_parity_to_f64(S.w, S.w32v, S.nrhs, vh, B->stream));
    // classical Gram-Schmidt, one or two passes (h1 = V^H w, w -= V h1, and again
    // with h2), then |w|^2
    d2_t* part = (d2_t*)S.partial.p;
    HIPCHK(launch_dot_b(S.V, (long long)N, k + 1, S.w, S.n, S.nrhs, part, S.nbx, h1, BLD, B->stream));
    HIPCHK(launch_update_b(S.w, S.V, (long long)N, k + 1, h1, BLD, -1.0, S.n, S.nrhs, B->stream));
    if (B->passes == 2) {
      HIPCHK(launch_dot_b(S.V, (long long)N, k + 1, S.w, S.n, S.nrhs, part, S.nbx, h2, BLD, B->stream));
      HIPCHK(launch_update_b(S.w, S.V, (long long)N, k + 1, h2, BLD, -1.0, S.n, S.nrhs, B->stream));
    }
    HIPCHK(launch_norm2_b(S.w, S.n, S.nrhs, (double*)part, S.nbx, hn, B->stream));
    // cycle mode: the next basis vector's factor 1/|w| on the device (0 after a
    // breakdown |w| <= 1e-14 and for right-hand sides that entered the cycle converged)
    if (B->cycle) HIPCHK(launch_inv_norm_b(hn, S.cf + cs, S.nrhs, 1e-28, B->stream));
  }
  return DDQ_OK;
}

// every pointer and value a captured step graph holds
std::vector<uintptr_t> batch_key(const ddq_batch* B, int m, int nu) {
  std::vector<uintptr_t> key{(uintptr_t)m, (uintptr_t)nu, (uintptr_t)B->sprec, (uintptr_t)B->passes,
                             (uintptr_t)B->cycle};
  for (const auto& S : B->sys) {
    const ddq_lattice* L = S.L;
    uint64_t om;
    std::memcpy(&om, &S.omega, 8);
    for (uintptr_t v : {(uintptr_t)S.w64.p, (uintptr_t)S.w32.p, (uintptr_t)S.small.p, (uintptr_t)S.partial.p, (uintptr_t)S.cyc.p,
                        (uintptr_t)L->tmp[DDQ_F32].p, (uintptr_t)L->tmp[B->sprec].p,
                        (uintptr_t)L->links[B->sprec][0], (uintptr_t)L->links[B->sprec][1],
                        (uintptr_t)L->clov[B->sprec][0], (uintptr_t)L->clov[B->sprec][1],
                        (uintptr_t)L->links[DDQ_F32][0], (uintptr_t)L->links[DDQ_F32][1],
                        (uintptr_t)L->clov[DDQ_F32][0], (uintptr_t)L->clov[DDQ_F32][1], (uintptr_t)L->link12,
                        (uintptr_t)om})
      key.push_back(v);
    const MrTile* t = L->tile_for(S.nrhs);
    key.push_back(t ? (uintptr_t)(1 + t->nb + 8 * t->g + 64 * t->xmap) : 0);
    key.push_back(t ? (uintptr_t)(t->passes + 16 * t->lds_kb) : 0);
  }
  return key;
}

int batch_capture(ddq_batch* B, int m, int nu) {
  std::vector<uintptr_t> key = batch_key(B, m, nu);
  if (key == B->graph_key) return DDQ_OK;
  batch_release_graphs(B);
  // per-step mode: one graph per step index; cycle mode: one graph of all m steps
  const int ngraph = B->cycle ? 1 : m;
  B->step_graph.assign(ngraph, nullptr);
  for (int k = 0; k < ngraph; ++k) {
    hipGraph_t g = nullptr;
    HIPCHK(hipStreamBeginCapture(B->stream, hipStreamCaptureModeThreadLocal));
    int r = DDQ_OK;
    for (int q = B->cycle ? 0 : k; q <= (B->cycle ? m - 1 : k) && r == DDQ_OK; ++q) r = batch_step(B, q, nu);
    hipError_t e = hipStreamEndCapture(B->stream, &g);
    if (r < 0 || e != hipSuccess) {
      if (g) (void)hipGraphDestroy(g);
      batch_release_graphs(B);
      if (r < 0) return r;
      HIPCHK(e);
    }
    e = hipGraphInstantiate(&B->step_graph[k], g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      batch_release_graphs(B);
      HIPCHK(e);
    }
  }
  B->graph_key = key;
  return DDQ_OK;
}

// the lattices run on the batch's stream, unprofiled, for the duration of a solve
struct LatticeStreamGuard {
  std::vector<std::pair<ddq_lattice*, std::pair<hipStream_t, bool>>> saved;
  LatticeStreamGuard(ddq_batch* B) {
    for (auto& S : B->sys) {
      saved.push_back({S.L, {S.L->stream, S.L->prof_on}});
      S.L->stream = B->stream;
      S.L->prof_on = false;
    }
  }
  ~LatticeStreamGuard() {
    for (auto it = saved.rbegin(); it != saved.rend(); ++it) {
      it->first->stream = it->second.first;
      it->first->prof_on = it->second.second;
    }
  }
};

struct RhsState {
  double bnorm = 0, target = 0, beta = 0, full = 0;
  bool active = false, stopped = true;
  int k_used = 0;
  std::vector<cd> g, y;
  std::vector<std::vector<cd>> R;
  std::vector<Givens> rot;
};

}  // namespace

extern "C" {

int ddq_batch_create(ddq_lattice* const* lats, const int* nrhs, int nlat, void* hip_stream, ddq_batch** out) {
  if (!out) return fail(DDQ_ERR_ARG, "out is null");
  *out = nullptr;
  if (!lats || !nrhs || nlat < 1) return fail(DDQ_ERR_ARG, "need at least one lattice");
  for (int l = 0; l < nlat; ++l) {
    if (!lats[l] || nrhs[l] < 1) return fail(DDQ_ERR_ARG, "null lattice or nrhs < 1 in the batch");
    for (int q = 0; q < l; ++q)
      if (lats[q] == lats[l]) return fail(DDQ_ERR_ARG, "a lattice appears twice in the batch");
  }
  ddq_batch* B = new ddq_batch();
  B->user = (hipStream_t)hip_stream;
  hipError_t e = hipStreamCreateWithFlags(&B->stream, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&B->ev, hipEventDisableTiming);
  if (e != hipSuccess) {
    if (B->stream) (void)hipStreamDestroy(B->stream);
    delete B;
    HIPCHK(e);
  }
  for (int l = 0; l < nlat; ++l) {
    ddq_batch::Sys S;
    S.L = lats[l];
    S.nrhs = nrhs[l];
    S.n = lats[l]->nvec();
    long long nb = (S.n + 255) / 256;
    S.nbx = (int)(nb > 512 ? 512 : nb);
    B->sys.push_back(std::move(S));
  }
  *out = B;
  return DDQ_OK;
}

int ddq_batch_reserve(ddq_batch* B, int max_m, int cycle_graph) {
  if (!B) return fail(DDQ_ERR_ARG, "null batch");
  if (max_m < 1 || max_m > BLD - 1) return fail(DDQ_ERR_ARG, "max_m must be in [1, 127]");
  AllocScope scope;
  B->res_m = std::max(B->res_m, max_m);
  B->res_cycle = B->res_cycle || cycle_graph != 0;
  for (auto& S : B->sys) {
    CHK(check_ready(S.L, DDQ_F32));
    CHK(batch_workspace(S, B->res_m, B->res_cycle != 0));
    // u_o of nrhs right-hand sides in every stored precision (the 16-bit smoothers)
    S.L->res_nrhs = std::max(S.L->res_nrhs, S.nrhs);
    CHK(reserve_impl(S.L));
  }
  CHK(batch_host(B, std::max(batch_host_doubles(B, B->res_m, false), batch_host_doubles(B, B->res_m, B->res_cycle != 0)) * 8));
  // multi-right-hand-side tiles of lattices not tuned for their count yet
  for (auto& S : B->sys)
    if (S.nrhs > 1 && !S.L->tile_for(S.nrhs)) {
      const hipStream_t keep = S.L->stream;
      S.L->stream = B->stream;
      const int r = ddq_tune_multi_rhs(S.L, S.nrhs, 3, nullptr, 0, nullptr, nullptr);
      S.L->stream = keep;
      CHK(r);
    }
  HIPCHK(hipStreamSynchronize(B->stream));
  return DDQ_OK;
}

int ddq_batch_destroy(ddq_batch* B) {
  if (!B) return DDQ_OK;
  if (B->stream) (void)hipStreamSynchronize(B->stream);
  batch_release_graphs(B);
  for (auto& S : B->sys) {
    S.w64.release();
    S.w32.release();
    S.small.release();
    S.partial.release();
    S.cyc.release();
  }
  if (B->host) (void)hipHostFree(B->host);
  if (B->ev) (void)hipEventDestroy(B->ev);
  if (B->stream) (void)hipStreamDestroy(B->stream);
  delete B;
  return DDQ_OK;
}

int ddq_batch_solve(ddq_batch* B, void* const* x, const void* const* b, const ddq_gmres_params* P,
                    const double* omegas, ddq_solve_info* info) {
  auto t0 = std::chrono::steady_clock::now();
  if (!B || !x || !b || !P) return fail(DDQ_ERR_ARG, "batch, x, b and params must be non-null");
  const int m = P->m;
  if (m < 1 || m > BLD - 1) return fail(DDQ_ERR_ARG, "cycle length m must be in [1, 127]");
  if (P->inner_prec != DDQ_F32) return fail(DDQ_ERR_ARG, "the batched solver runs its inner stage in FP32");
  if (P->max_cycles < 0 || !(P->tol >= 0.0) || P->smoother_sweeps < 0)
    return fail(DDQ_ERR_ARG, "bad max_cycles, tol or smoother_sweeps");
  const int nu = P->smoother_sweeps;
  const double red = P->inner_reduction > 0.0 ? P->inner_reduction : 1e-5;
  const int ns = (int)B->sys.size();
  const int sprec = is16(P->smoother_prec) ? P->smoother_prec : DDQ_F32;
  if (P->orth_passes < 0 || P->orth_passes > 2) return fail(DDQ_ERR_ARG, "orth_passes must be 0, 1 or 2");
  const int cycle = P->cycle_graph ? 1 : 0;
  // pinned host layout: per system, the D2H block then the H2D block
  std::vector<size_t> d2h(ns), h2d(ns);
  size_t host_doubles = 0;
  for (int s = 0; s < ns; ++s) {
    auto& S = B->sys[s];
    CHK(check_ready(S.L, DDQ_F32));
    if (sprec != DDQ_F32) CHK(check_ready(S.L, sprec));
    if (!x[s] || !b[s] || x[s] == b[s]) return fail(DDQ_ERR_ARG, "bad x / b pointers in the batch");
    S.omega = omegas ? omegas[s] : P->omega;
    if (nu > 0 && !(std::isfinite(S.omega) && S.omega > 0.0)) return fail(DDQ_ERR_ARG, "omega must be positive");
    d2h[s] = host_doubles;
    host_doubles += batch_d2h_bytes(S.nrhs, cycle ? m : 1) / 8;
    h2d[s] = host_doubles;
    host_doubles += batch_h2d_doubles(S.nrhs);
  }
  if (m > B->res_m || (cycle && !B->res_cycle))
    return fail(DDQ_ERR_STATE, "the batch's work space is reserved for m <= " + std::to_string(B->res_m) +
                                   (B->res_cycle ? " (cycle mode included)" : " (step mode)") + ": call ddq_batch_reserve");
  CHK(batch_host(B, host_doubles * 8));
  // order after the caller's stream, then run on the batch's own
  HIPCHK(hipEventRecord(B->ev, B->user));
  HIPCHK(hipStreamWaitEvent(B->stream, B->ev, 0));
  LatticeStreamGuard guard(B);
  B->sprec = sprec;
  B->passes = P->orth_passes == 1 ? 1 : 2;
  B->cycle = cycle;
  for (auto& S : B->sys) {
    CHK(batch_workspace(S, m, cycle));
    if (sprec != DDQ_F32) CHK(ensure_tmp(S.L, sprec, S.nrhs));
  }

  std::vector<std::vector<RhsState>> st(ns);
  int iters = 0, cycles = 0;
  auto fetch_norms = [&](int s) -> int {  // S.hn -> host D2H block of system s
    auto& S = B->sys[s];
    HIPCHK(hipMemcpyAsync(B->host + d2h[s], S.hn, S.nrhs * 8, hipMemcpyDeviceToHost, B->stream));
    return DDQ_OK;
  };
  auto push = [&](int s, void* dst, size_t off, size_t bytes) -> int {  // host H2D block of system s -> dst
    HIPCHK(hipMemcpyAsync(dst, B->host + h2d[s] + off, bytes, hipMemcpyHostToDevice, B->stream));
    return DDQ_OK;
  };
  // |b| per right-hand side (full vectors: 2n complex each), eq. 2 prepare, x_e
  for (int s = 0; s < ns; ++s) {
    auto& S = B->sys[s];
    HIPCHK(launch_norm2_b((const d2_t*)b[s], 2 * S.n, S.nrhs, (double*)S.partial.p, S.nbx, S.hn, B->stream));
    CHK(fetch_norms(s));
    CHK(prepare_impl(S.L, S.nrhs, (const d2_t*)b[s], S.bt, S.w));
    HIPCHK(launch_pack_parity<double>(S.L->geo, 0, S.nrhs, (const d2_t*)x[s], S.xe, B->stream));
  }
  HIPCHK(hipStreamSynchronize(B->stream));
  for (int s = 0; s < ns; ++s) {
    auto& S = B->sys[s];
    st[s].resize(S.nrhs);
    for (int r = 0; r < S.nrhs; ++r) {
      auto& R = st[s][r];
      R.bnorm = std::sqrt(B->host[d2h[s] + r]);
      if (!std::isfinite(R.bnorm)) return fail(DDQ_ERR_NONFINITE, "right-hand side is not finite");
      R.target = P->tol * R.bnorm;
      R.g.assign(m + 2, 0.0);
      R.y.assign(m + 1, 0.0);
      R.R.assign(m, std::vector<cd>(m + 1));
      R.rot.assign(m, Givens{1.0, 0.0});
    }
  }
  CHK(batch_capture(B, m, nu));

  bool all_done = false;
  cycles = 0;
  for (;;) {  // restarts, then eq. 2's reconstruction and the full residuals
  for (;; ++cycles) {
    // FP64 residuals (the refinement step) and their norms
    for (int s = 0; s < ns; ++s) {
      auto& S = B->sys[s];
      CHK(resid<double>(S.L, DDQ_F64, S.nrhs, S.xe, S.bt, S.V));
      HIPCHK(launch_norm2_b(S.V, S.n, S.nrhs, (double*)S.partial.p, S.nbx, S.hn, B->stream));
      CHK(fetch_norms(s));
    }
    HIPCHK(hipStreamSynchronize(B->stream));
    all_done = true;
    for (int s = 0; s < ns; ++s) {
      auto& S = B->sys[s];
      for (int r = 0; r < S.nrhs; ++r) {
        auto& R = st[s][r];
        R.beta = std::sqrt(B->host[d2h[s] + r]);
        if (!std::isfinite(R.beta)) return fail(DDQ_ERR_NONFINITE, "residual norm is not finite");
        R.active = R.beta > R.target;
        R.stopped = !R.active;
        R.k_used = 0;
        if (R.active) all_done = false;
      }
    }
    if (all_done || cycles == P->max_cycles) break;
    // v_0 = r / beta; converged systems get a zero basis (factor 0) for the cycle
    for (int s = 0; s < ns; ++s) {
      auto& S = B->sys[s];
      double* fh = B->host + h2d[s] + 2 * BLD * S.nrhs;
      for (int r = 0; r < S.nrhs; ++r) {
        auto& R = st[s][r];
        fh[r] = R.active ? 1.0 / R.beta : 0.0;
        std::fill(R.g.begin(), R.g.end(), cd(0.0));
        R.g[0] = R.beta;
      }
      CHK(push(s, S.f, 2 * BLD * S.nrhs, S.nrhs * 8));
      HIPCHK(launch_scale_b(S.V, S.V, S.f, S.n, S.nrhs, B->stream));
    }
    // Givens update of right-hand side R with Hessenberg column k (h1 + h2, |w| = nrm);
    // returns false on a non-finite norm
    auto column = [&](RhsState& R, int k, const double* h1, const double* h2, double nrm) -> bool {
      if (!std::isfinite(nrm)) return false;
      std::vector<cd> col(k + 2);
      for (int j = 0; j <= k; ++j)
        col[j] = h2 ? cd(h1[2 * j] + h2[2 * j], h1[2 * j + 1] + h2[2 * j + 1]) : cd(h1[2 * j], h1[2 * j + 1]);
      col[k + 1] = nrm;
      for (int j = 0; j < k; ++j) {
        cd t = R.rot[j].c * col[j] + R.rot[j].s * col[j + 1];
        col[j + 1] = -std::conj(R.rot[j].s) * col[j] + R.rot[j].c * col[j + 1];
        col[j] = t;
      }
      R.rot[k] = make_givens(col[k], col[k + 1]);
      col[k] = R.rot[k].c * col[k] + R.rot[k].s * col[k + 1];
      R.g[k + 1] = -std::conj(R.rot[k].s) * R.g[k];
      R.g[k] = R.rot[k].c * R.g[k];
      for (int j = 0; j <= k; ++j) R.R[k][j] = col[j];
      R.k_used = k + 1;
      return true;
    };
    if (cycle) {
      // the whole cycle is one graph of m steps (basis factors on the device); the
      // host reads every step's coefficients once and, per right-hand side, takes the
      // columns up to the first whose estimate meets the cycle target (or a
      // breakdown): the update the step-by-step mode makes, the later steps unused
      HIPCHK(hipGraphLaunch(B->step_graph[0], B->stream));
      for (int s = 0; s < ns; ++s)
        HIPCHK(hipMemcpyAsync(B->host + d2h[s], B->sys[s].ch1, batch_d2h_bytes(B->sys[s].nrhs, m),
                              hipMemcpyDeviceToHost, B->stream));
      HIPCHK(hipStreamSynchronize(B->stream));
      iters += m;
      for (int s = 0; s < ns; ++s) {
        auto& S = B->sys[s];
        const size_t mr = (size_t)m * S.nrhs;
        const double* c1 = B->host + d2h[s];
        const double* c2 = c1 + mr * BLD * 2;
        const double* cn = c2 + mr * BLD * 2;
        for (int r = 0; r < S.nrhs; ++r) {
          auto& R = st[s][r];
          if (!R.active) continue;
          for (int k = 0; k < m; ++k) {
            const size_t slot = (size_t)k * S.nrhs + r;
            const double nrm = std::sqrt(cn[slot]);
            if (!column(R, k, c1 + slot * BLD * 2, B->passes == 2 ? c2 + slot * BLD * 2 : nullptr, nrm))
              return fail(DDQ_ERR_NONFINITE, "Arnoldi norm is not finite");
            // breakdown: the device zeroed the later basis vectors
            if (std::abs(R.g[k + 1]) <= std::max(R.target, red * R.beta) || nrm <= 1e-14) break;
          }
        }
      }
    }
    for (int k = 0; k < m && !cycle; ++k) {
      HIPCHK(hipGraphLaunch(B->step_graph[k], B->stream));
      for (int s = 0; s < ns; ++s)
        HIPCHK(hipMemcpyAsync(B->host + d2h[s], B->sys[s].h1, batch_d2h_bytes(B->sys[s].nrhs),
                              hipMemcpyDeviceToHost, B->stream));
      HIPCHK(hipStreamSynchronize(B->stream));  // one synchronisation for the whole batch
      ++iters;
      bool any_running = false;
      for (int s = 0; s < ns; ++s) {
        auto& S = B->sys[s];
        const double* hh = B->host + d2h[s];
        const double* hn = hh + (size_t)S.nrhs * 2 * BLD * 2;
        double* fh = B->host + h2d[s] + 2 * BLD * S.nrhs;
        for (int r = 0; r < S.nrhs; ++r) {
          auto& R = st[s][r];
          fh[r] = 0.0;
          if (R.stopped) continue;
          const double* h1 = hh + (size_t)r * BLD * 2;
          const double* h2 = hh + ((size_t)S.nrhs + r) * BLD * 2;
          const double nrm = std::sqrt(hn[r]);
          if (!column(R, k, h1, B->passes == 2 ? h2 : nullptr, nrm))
            return fail(DDQ_ERR_NONFINITE, "Arnoldi norm is not finite");
          if (std::abs(R.g[k + 1]) <= std::max(R.target, red * R.beta) || nrm <= 1e-14 * R.beta) {
            R.stopped = true;
          } else {
            fh[r] = 1.0 / nrm;
            any_running = true;
          }
        }
      }
      if (!any_running || k + 1 == m) break;
      // factors of v_{k+1} = w / |w|, applied inside the next step's graph;
      // stopped right-hand sides continue on zero vectors
      for (int s = 0; s < ns; ++s) CHK(push(s, B->sys[s].f, 2 * BLD * B->sys[s].nrhs, B->sys[s].nrhs * 8));
    }
    // y = R^-1 g per right-hand side (zero beyond its own k_used); x_e += Z y
    for (int s = 0; s < ns; ++s) {
      auto& S = B->sys[s];
      double* yh = B->host + h2d[s];
      std::fill(yh, yh + (size_t)S.nrhs * BLD * 2, 0.0);
      int kmax = 0;
      for (int r = 0; r < S.nrhs; ++r) {
        auto& R = st[s][r];
        if (!R.active || R.k_used == 0) continue;
        for (int j = R.k_used - 1; j >= 0; --j) {
          cd sum = R.g[j];
          for (int q = j + 1; q < R.k_used; ++q) sum -= R.R[q][j] * R.y[q];
          R.y[j] = sum / R.R[j][j];
        }
        for (int j = 0; j < R.k_used; ++j) {
          yh[((size_t)r * BLD + j) * 2] = R.y[j].real();
          yh[((size_t)r * BLD + j) * 2 + 1] = R.y[j].imag();
        }
        kmax = std::max(kmax, R.k_used);
      }
      if (kmax == 0) continue;
      CHK(push(s, S.y, 0, (size_t)S.nrhs * BLD * 16));
      HIPCHK(launch_update_b(S.xe, S.Z, (long long)S.nrhs * S.n, kmax, S.y, BLD, 1.0, S.n, S.nrhs, B->stream));
    }
  }
  // eq. 2 reconstruction (x_o in S.z), then |b - D x| in FP64 per system: the Schur
  // residual and the full one agree in exact arithmetic; a system whose full residual
  // misses tol |b| gets its Schur target lowered by the observed ratio and the restarts
  // continue, so DDQ_OK always means the full bar
  for (auto& S : B->sys) {
    const int s = (int)(&S - B->sys.data());
    CHK(reconstruct_impl(S.L, S.nrhs, S.xe, (const d2_t*)b[s], (d2_t*)x[s], S.w, S.z));
  }
  bool retry = false;
  for (int s = 0; s < ns; ++s) {
    auto& S = B->sys[s];
    for (int r = 0; r < S.nrhs; ++r) {
      auto& R = st[s][r];
      const size_t o = (size_t)r * S.n;
      CHK(full_residual_norm(S.L, S.xe + o, S.z + o, (const d2_t*)b[s] + 2 * o, S.V, S.V + S.n, &R.full));
      if (!std::isfinite(R.full)) return fail(DDQ_ERR_NONFINITE, "full residual norm is not finite");
      if (R.full > P->tol * R.bnorm) {
        retry = true;
        R.target = std::min(0.5 * R.target, 0.9 * R.beta * P->tol * R.bnorm / R.full);
      }
    }
  }
  if (!all_done) break;
  if (!retry) break;
  if (cycles >= P->max_cycles) {
    all_done = false;
    break;
  }
  }
  HIPCHK(hipStreamSynchronize(B->stream));
  const double ms = std::chrono::duration<double, std::milli>(std::chrono::steady_clock::now() - t0).count();
  if (info) {
    int idx = 0;
    for (int s = 0; s < ns; ++s)
      for (int r = 0; r < B->sys[s].nrhs; ++r, ++idx) {
        const auto& R = st[s][r];
        info[idx].cycles = cycles;
        info[idx].iters = iters;
        info[idx].applies_f64 = cycles + 1;
        info[idx].applies_lo = iters * (nu > 0 ? nu : 1);
        info[idx].true_relres = R.bnorm > 0 ? R.full / R.bnorm : 0.0;
        info[idx].t_total_ms = ms;
      }
  }
  if (!all_done) {
    g_err = "batched GMRES stopped at max_cycles";
    return DDQ_NOT_CONVERGED;
  }
  return DDQ_OK;
}

}  // extern "C"
