// fields.hip -- set-up kernels: gauge packing, clover blocks and their inverses,
// parity packing of vectors.
#include "ddq_internal.h"

namespace ddq {

// lexicographic index of coordinates (x, y, z, t)
__device__ __forceinline__ long long lex(const Geo& g, int x, int y, int z, int t) {
  return x + (long long)g.L[0] * (y + (long long)g.L[1] * (z + (long long)g.L[2] * t));
}

__device__ __forceinline__ void coords_shift(const Geo& g, int c[4], int mu, int step) {
  c[mu] += step;
  if (c[mu] < 0) c[mu] += g.L[mu];
  if (c[mu] >= g.L[mu]) c[mu] -= g.L[mu];
}

// ---------------------------------------------------------------------------
// gauge packing: per parity p, direction mu and site i, complex rows 0..8 = U_mu(x)
// and rows 9..17 = U_mu(x-mu)^H (FP64: one complex per 16-byte element)
// ---------------------------------------------------------------------------
__global__ void k_pack_gauge(Geo g, const d2_t* __restrict__ U, d2_t* __restrict__ out_e,
                             d2_t* __restrict__ out_o) {
  const int vh = g.Vh;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 2LL * vh) return;
  const int p = (int)(tid / vh);
  const int i = (int)(tid % vh);
  Site s = decode(g, i, p);
  d2_t* out = p == 0 ? out_e : out_o;
  const long long n = lex(g, s.x, s.y, s.z, s.t);
  const size_t fsz = (size_t)LINK_ROWS * field_vh(vh);  // one direction's link field
  for (int mu = 0; mu < 4; ++mu) {
    const d2_t* u = U + (n * 4 + mu) * 9;
    for (int e = 0; e < 9; ++e) {
      out[mu * fsz + fidx(e, i, LINK_ROWS, vh)] = u[e];
      store_fence();
    }
    int c[4] = {s.x, s.y, s.z, s.t};
    coords_shift(g, c, mu, -1);
    const long long nb = lex(g, c[0], c[1], c[2], c[3]);
    const d2_t* ub = U + (nb * 4 + mu) * 9;
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        d2_t v = ub[3 * b + a];
        v.y = -v.y;
        out[mu * fsz + fidx(9 + 3 * a + b, i, LINK_ROWS, vh)] = v;
        store_fence();
      }
  }
}

hipError_t launch_pack_gauge_f64(const Geo& g, const d2_t* U, d2_t* out_e, d2_t* out_o, hipStream_t s) {
  long long n = 2LL * g.Vh;
  int blocks = (int)((n + 255) / 256);
  hipLaunchKernelGGL(k_pack_gauge, dim3(blocks), dim3(256), 0, s, g, U, out_e, out_o);
  return hipGetLastError();
}

// FP64 blocked fields (nfields fields of crows complex rows) -> FP32 blocked fields
// whose 16-byte element e holds complex rows 2e and 2e+1
__global__ void k_field_to_f32(const d2_t* __restrict__ in, f4_t* __restrict__ out, int nfields, int crows, int vh) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int er = crows / 2;
  const long long total = (long long)nfields * er * vh;
  if (tid >= total) return;
  const int i = (int)(tid % vh);
  const int e = (int)((tid / vh) % er);
  const int f = (int)(tid / ((long long)vh * er));
  const size_t fv = (size_t)field_vh(vh);
  const d2_t* src = in + (size_t)f * crows * fv;
  d2_t a = src[fidx(2 * e, i, crows, vh)], b = src[fidx(2 * e + 1, i, crows, vh)];
  f4_t o;
  o.x = (float)a.x;
  o.y = (float)a.y;
  o.z = (float)b.x;
  o.w = (float)b.y;
  out[(size_t)f * er * fv + fidx(e, i, er, vh)] = o;
}

// FP64 link fields (4 directions x LINK_ROWS) -> FP32 12-real link fields: complex
// rows 0..5 (first two rows of U_mu(x)) and 9..14 (of U_mu(x - mu)^H), paired
__global__ void k_links_to_f32_12(const d2_t* __restrict__ in, f4_t* __restrict__ out, int vh) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const int er = LINK12_ROWS / 2;
  if (tid >= 4LL * er * vh) return;
  const int i = (int)(tid % vh);
  const int e = (int)((tid / vh) % er);
  const int mu = (int)(tid / ((long long)vh * er));
  const size_t fv = (size_t)field_vh(vh);
  const d2_t* src = in + (size_t)mu * LINK_ROWS * fv;
  auto row = [](int k) { return k < 6 ? k : k + 3; };  // 12-real row -> 18-entry row
  d2_t a = src[fidx(row(2 * e), i, LINK_ROWS, vh)], b = src[fidx(row(2 * e + 1), i, LINK_ROWS, vh)];
  f4_t o;
  o.x = (float)a.x;
  o.y = (float)a.y;
  o.z = (float)b.x;
  o.w = (float)b.y;
  out[(size_t)mu * er * fv + fidx(e, i, er, vh)] = o;
}

hipError_t launch_links_to_f32_12(const d2_t* in, void* out, int vh, hipStream_t s) {
  const long long total = 4LL * (LINK12_ROWS / 2) * vh;
  hipLaunchKernelGGL(k_links_to_f32_12, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, in, (f4_t*)out, vh);
  return hipGetLastError();
}

hipError_t launch_field_to_f32(const d2_t* in, void* out, int nfields, int crows, int vh, hipStream_t s) {
  const long long total = (long long)nfields * (crows / 2) * vh;
  hipLaunchKernelGGL(k_field_to_f32, dim3((unsigned)((total + 255) / 256)), dim3(256), 0, s, in, (f4_t*)out,
                     nfields, crows, vh);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// clover blocks
// ---------------------------------------------------------------------------
struct M3 {
  cpx<double> a[3][3];
};

__device__ __forceinline__ M3 load_link(const Geo& g, const d2_t* U, const int c[4], int mu) {
  const long long n = lex(g, c[0], c[1], c[2], c[3]);
  const d2_t* u = U + (n * 4 + mu) * 9;
  M3 m;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      d2_t v = u[3 * a + b];
      m.a[a][b] = {v.x, v.y};
    }
  return m;
}

__device__ __forceinline__ M3 mul(const M3& A, const M3& B) {
  M3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cpx<double> s = A.a[a][0] * B.a[0][b];
      cfma(s, A.a[a][1], B.a[1][b]);
      cfma(s, A.a[a][2], B.a[2][b]);
      C.a[a][b] = s;
    }
  return C;
}

__device__ __forceinline__ M3 dagger(const M3& A) {
  M3 C;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) C.a[a][b] = conj(A.a[b][a]);
  return C;
}

// Q_munu(x): the four counter-clockwise leaves of the mu-nu plane that touch x
__device__ M3 clover_leaves(const Geo& g, const d2_t* U, const int x[4], int mu, int nu) {
  int c[4];
  M3 Q;
  // leaf 1: U_mu(x) U_nu(x+mu) U_mu(x+nu)^H U_nu(x)^H
  {
    M3 a = load_link(g, U, x, mu);
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, mu, 1);
    M3 b = load_link(g, U, c, nu);
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, nu, 1);
    M3 d = dagger(load_link(g, U, c, mu));
    M3 e = dagger(load_link(g, U, x, nu));
    Q = mul(mul(mul(a, b), d), e);
  }
  // leaf 2: U_nu(x) U_mu(x-mu+nu)^H U_nu(x-mu)^H U_mu(x-mu)
  {
    M3 a = load_link(g, U, x, nu);
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, mu, -1);
    coords_shift(g, c, nu, 1);
    M3 b = dagger(load_link(g, U, c, mu));
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, mu, -1);
    M3 d = dagger(load_link(g, U, c, nu));
    M3 e = load_link(g, U, c, mu);
    M3 L = mul(mul(mul(a, b), d), e);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q.a[i][j] = Q.a[i][j] + L.a[i][j];
  }
  // leaf 3: U_mu(x-mu)^H U_nu(x-mu-nu)^H U_mu(x-mu-nu) U_nu(x-nu)
  {
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, mu, -1);
    M3 a = dagger(load_link(g, U, c, mu));
    coords_shift(g, c, nu, -1);
    M3 b = dagger(load_link(g, U, c, nu));
    M3 d = load_link(g, U, c, mu);
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, nu, -1);
    M3 e = load_link(g, U, c, nu);
    M3 L = mul(mul(mul(a, b), d), e);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q.a[i][j] = Q.a[i][j] + L.a[i][j];
  }
  // leaf 4: U_nu(x-nu)^H U_mu(x-nu) U_nu(x+mu-nu) U_mu(x)^H
  {
    for (int k = 0; k < 4; ++k) c[k] = x[k];
    coords_shift(g, c, nu, -1);
    M3 a = dagger(load_link(g, U, c, nu));
    M3 b = load_link(g, U, c, mu);
    coords_shift(g, c, mu, 1);
    M3 d = load_link(g, U, c, nu);
    M3 e = dagger(load_link(g, U, x, mu));
    M3 L = mul(mul(mul(a, b), d), e);
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) Q.a[i][j] = Q.a[i][j] + L.a[i][j];
  }
  return Q;
}

// F = (Q - Q^H) / 8
__device__ __forceinline__ M3 field_from_leaves(const M3& Q) {
  M3 F;
  for (int a = 0; a < 3; ++a)
    for (int b = 0; b < 3; ++b) {
      cpx<double> q = Q.a[a][b], qt = conj(Q.a[b][a]);
      F.a[a][b] = {(q.r - qt.r) * 0.125, (q.i - qt.i) * 0.125};
    }
  return F;
}

// write a Hermitian 6x6 block (full matrix M) into the packed 18-slot format
// block blk of site i of a 36-row clover field
__device__ __forceinline__ void store_packed(d2_t* C, int blk, int i, int vh, const cpx<double> M[6][6]) {
  for (int k = 0; k < 3; ++k) {
    d2_t v;
    v.x = M[2 * k][2 * k].r;
    v.y = M[2 * k + 1][2 * k + 1].r;
    C[fidx(18 * blk + k, i, 36, vh)] = v;
    store_fence();
  }
  for (int j = 0; j < 6; ++j)
    for (int k = j + 1; k < 6; ++k) {
      d2_t v;
      v.x = M[j][k].r;
      v.y = M[j][k].i;
      C[fidx(18 * blk + tri_slot(j, k), i, 36, vh)] = v;
      store_fence();
    }
}

// In-place inverse of a Hermitian positive-definite 6x6 matrix by Cholesky
// A = L L^H; returns false if a pivot is not positive.
__device__ bool hpd_inverse6(cpx<double> A[6][6]) {
  cpx<double> L[6][6];
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) L[j][k] = {0.0, 0.0};
  for (int j = 0; j < 6; ++j) {
    double d = A[j][j].r;
    for (int k = 0; k < j; ++k) d -= L[j][k].r * L[j][k].r + L[j][k].i * L[j][k].i;
    if (!(d > 0.0)) return false;
    double ljj = sqrt(d);
    L[j][j] = {ljj, 0.0};
    for (int r = j + 1; r < 6; ++r) {
      cpx<double> s = A[r][j];
      for (int k = 0; k < j; ++k) {
        cpx<double> t = L[r][k] * conj(L[j][k]);
        s = s - t;
      }
      L[r][j] = {s.r / ljj, s.i / ljj};
    }
  }
  // Linv = L^-1 (lower triangular), column by column by forward substitution
  cpx<double> Li[6][6];
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) Li[j][k] = {0.0, 0.0};
  for (int c = 0; c < 6; ++c) {
    Li[c][c] = {1.0 / L[c][c].r, 0.0};
    for (int r = c + 1; r < 6; ++r) {
      cpx<double> s = {0.0, 0.0};
      for (int k = c; k < r; ++k) cfma(s, L[r][k], Li[k][c]);
      Li[r][c] = {-s.r / L[r][r].r, -s.i / L[r][r].r};
    }
  }
  // A^-1 = Li^H Li
  for (int j = 0; j < 6; ++j)
    for (int k = 0; k < 6; ++k) {
      cpx<double> s = {0.0, 0.0};
      for (int r = (j > k ? j : k); r < 6; ++r) cfma_conj(s, Li[r][j], Li[r][k]);
      A[j][k] = s;
    }
  return true;
}

// Per site: A_+- = (4 + m0) 1_6 + (i c_sw / 2) sum_l s_l (x) E_l^+-,
// E_l^+- = +-F_{l t} - F_{jk}, (l, j, k) cyclic over (x, y, z).  This is the
// chiral-basis form of (4 + m0) + (i c_sw / 4) sum sigma_munu F_munu:
// sigma_{l t} = diag(s_l, -s_l) and sigma_{jk} = -diag(s_l, s_l).
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1))) k_clover_build(Geo g, const d2_t* __restrict__ U, double c_sw, double m0,
                               d2_t* __restrict__ cl_e, d2_t* __restrict__ cl_o_inv,
                               d2_t* __restrict__ cl_o, int* notpd) {
  const int vh = g.Vh;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 2LL * vh) return;
  const int p = (int)(tid / vh);
  const int i = (int)(tid % vh);
  Site s = decode(g, i, p);
  const int x[4] = {s.x, s.y, s.z, s.t};
  // the six F_munu, indexed by (mu, nu) with mu < nu
  M3 Fxt = field_from_leaves(clover_leaves(g, U, x, 0, 3));
  M3 Fyt = field_from_leaves(clover_leaves(g, U, x, 1, 3));
  M3 Fzt = field_from_leaves(clover_leaves(g, U, x, 2, 3));
  M3 Fyz = field_from_leaves(clover_leaves(g, U, x, 1, 2));
  M3 Fzx;  // F_zx = -F_xz
  {
    M3 Fxz = field_from_leaves(clover_leaves(g, U, x, 0, 2));
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) Fzx.a[a][b] = {-Fxz.a[a][b].r, -Fxz.a[a][b].i};
  }
  M3 Fxy = field_from_leaves(clover_leaves(g, U, x, 0, 1));
  const double h = 0.5 * c_sw;
  for (int blk = 0; blk < 2; ++blk) {
    const double sg = blk == 0 ? 1.0 : -1.0;
    cpx<double> E[3][3][3];  // E_l
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        E[0][a][b] = sg * Fxt.a[a][b] - Fyz.a[a][b];
        E[1][a][b] = sg * Fyt.a[a][b] - Fzx.a[a][b];
        E[2][a][b] = sg * Fzt.a[a][b] - Fxy.a[a][b];
      }
    // M = (i h) [s1 (x) E0 + s2 (x) E1 + s3 (x) E2] + (4 + m0)
    cpx<double> M[6][6];
    for (int a = 0; a < 3; ++a)
      for (int b = 0; b < 3; ++b) {
        cpx<double> e0 = E[0][a][b], e1 = E[1][a][b], e2 = E[2][a][b];
        // spin blocks of s1 e0 + s2 e1 + s3 e2: [[e2, e0 - i e1], [e0 + i e1, -e2]]
        cpx<double> b00 = e2, b11 = {-e2.r, -e2.i};
        cpx<double> b01 = e0 - times_i(e1), b10 = e0 + times_i(e1);
        M[a][b] = h * times_i(b00);
        M[a][3 + b] = h * times_i(b01);
        M[3 + a][b] = h * times_i(b10);
        M[3 + a][3 + b] = h * times_i(b11);
      }
    for (int k = 0; k < 6; ++k) M[k][k].r += 4.0 + m0;
    if (p == 0) {
      store_packed(cl_e, blk, i, vh, M);
    } else {
      if (cl_o) store_packed(cl_o, blk, i, vh, M);  // A_oo itself, for the full operator
      if (!hpd_inverse6(M)) {
        *notpd = 1;
        for (int j = 0; j < 6; ++j)
          for (int k = 0; k < 6; ++k) M[j][k] = {0.0, 0.0};
      }
      store_packed(cl_o_inv, blk, i, vh, M);
    }
  }
}

hipError_t launch_clover_build(const Geo& g, const d2_t* U, double c_sw, double m0, d2_t* cl_e,
                               d2_t* cl_o_inv, d2_t* cl_o, int* notpd, hipStream_t s) {
  long long n = 2LL * g.Vh;
  int blocks = (int)((n + 127) / 128);
  hipLaunchKernelGGL(k_clover_build, dim3(blocks), dim3(128), 0, s, g, U, c_sw, m0, cl_e, cl_o_inv, cl_o,
                     notpd);
  return hipGetLastError();
}

// packed [2][18][vh] -> dense [vh][2][6][6]
__global__ void k_clover_export(Geo g, const d2_t* __restrict__ P, d2_t* __restrict__ D) {
  const int vh = g.Vh;
  long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 2LL * vh) return;
  const int blk = (int)(tid / vh);
  const int i = (int)(tid % vh);
  d2_t* out = D + ((size_t)i * 2 + blk) * 36;
  for (int k = 0; k < 3; ++k) {
    d2_t d = P[fidx(18 * blk + k, i, 36, vh)];
    d2_t a, b;
    a.x = d.x; a.y = 0.0;
    b.x = d.y; b.y = 0.0;
    out[(2 * k) * 6 + 2 * k] = a;
    out[(2 * k + 1) * 6 + 2 * k + 1] = b;
    store_fence();
  }
  for (int j = 0; j < 6; ++j)
    for (int k = j + 1; k < 6; ++k) {
      d2_t v = P[fidx(18 * blk + tri_slot(j, k), i, 36, vh)];
      out[j * 6 + k] = v;
      store_fence();
      v.y = -v.y;
      out[k * 6 + j] = v;
      store_fence();
    }
}

hipError_t launch_clover_export(const Geo& g, const d2_t* packed, d2_t* dense, hipStream_t s) {
  long long n = 2LL * g.Vh;
  hipLaunchKernelGGL(k_clover_export, dim3((int)((n + 255) / 256)), dim3(256), 0, s, g, packed, dense);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// parity packing of vectors: full [n][12] <-> parity layout (FP64: [12][vh]
// complex128; FP32: [6][vh] elements of two complex64, rows 2k and 2k+1)
// ---------------------------------------------------------------------------
template <typename R>
__global__ void k_pack_parity(Geo g, int parity, const pair<R>* __restrict__ full, pair<R>* __restrict__ v) {
  const int vh = g.Vh;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  const size_t r = blockIdx.y;
  Site s = decode(g, i, parity);
  const long long n = lex(g, s.x, s.y, s.z, s.t);
  const pair<R>* src = full + r * (size_t)2 * vh * 12 + n * 12;
  pair<R>* dst = v + r * (size_t)vh * 12;
  constexpr int C = CPE<R>;
  for (int k = 0; k < 12; ++k) {
    dst[((size_t)(k / C) * vh + i) * C + (k % C)] = src[k];
    store_fence();
  }
}

template <typename R>
__global__ void k_unpack_parity(Geo g, int parity, const pair<R>* __restrict__ v, pair<R>* __restrict__ full) {
  const int vh = g.Vh;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= vh) return;
  const size_t r = blockIdx.y;
  Site s = decode(g, i, parity);
  const long long n = lex(g, s.x, s.y, s.z, s.t);
  pair<R>* dst = full + r * (size_t)2 * vh * 12 + n * 12;
  const pair<R>* src = v + r * (size_t)vh * 12;
  constexpr int C = CPE<R>;
  for (int k = 0; k < 12; ++k) {
    dst[k] = src[((size_t)(k / C) * vh + i) * C + (k % C)];
    store_fence();
  }
}

template <typename R>
hipError_t launch_pack_parity(const Geo& g, int parity, int nrhs, const pair<R>* full, pair<R>* v,
                              hipStream_t s) {
  dim3 grid((g.Vh + 255) / 256, nrhs);
  hipLaunchKernelGGL((k_pack_parity<R>), grid, dim3(256), 0, s, g, parity, full, v);
  return hipGetLastError();
}

template <typename R>
hipError_t launch_unpack_parity(const Geo& g, int parity, int nrhs, const pair<R>* v, pair<R>* full,
                                hipStream_t s) {
  dim3 grid((g.Vh + 255) / 256, nrhs);
  hipLaunchKernelGGL((k_unpack_parity<R>), grid, dim3(256), 0, s, g, parity, v, full);
  return hipGetLastError();
}

template hipError_t launch_pack_parity<double>(const Geo&, int, int, const d2_t*, d2_t*, hipStream_t);
template hipError_t launch_pack_parity<float>(const Geo&, int, int, const f2_t*, f2_t*, hipStream_t);
template hipError_t launch_unpack_parity<double>(const Geo&, int, int, const d2_t*, d2_t*, hipStream_t);
template hipError_t launch_unpack_parity<float>(const Geo&, int, int, const f2_t*, f2_t*, hipStream_t);

// FP64 parity vectors [nrhs][12][vh] <-> FP32 parity vectors [nrhs][6][vh][2]
__global__ void k_parity_to_f32(f4_t* __restrict__ y, const d2_t* __restrict__ x, long long n6, int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;  // (rhs, k, i)
  if (t >= n6) return;
  const int i = (int)(t % vh);
  const long long rk = t / vh;  // rhs * 6 + k
  const long long rhs = rk / 6;
  const int k = (int)(rk % 6);
  const d2_t* xr = x + rhs * 12LL * vh;
  d2_t a = xr[(size_t)(2 * k) * vh + i], b = xr[(size_t)(2 * k + 1) * vh + i];
  f4_t o;
  o.x = (float)a.x;
  o.y = (float)a.y;
  o.z = (float)b.x;
  o.w = (float)b.y;
  y[t] = o;
}

__global__ void k_parity_to_f64(d2_t* __restrict__ y, const f4_t* __restrict__ x, long long n6, int vh) {
  const long long t = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (t >= n6) return;
  const int i = (int)(t % vh);
  const long long rk = t / vh;
  const long long rhs = rk / 6;
  const int k = (int)(rk % 6);
  d2_t* yr = y + rhs * 12LL * vh;
  f4_t q = x[t];
  d2_t a, b;
  a.x = q.x;
  a.y = q.y;
  b.x = q.z;
  b.y = q.w;
  yr[(size_t)(2 * k) * vh + i] = a;
  store_fence();
  yr[(size_t)(2 * k + 1) * vh + i] = b;
}

hipError_t launch_parity_to_f32(void* y, const d2_t* x, int nrhs, int vh, hipStream_t s) {
  const long long n6 = 6LL * vh * nrhs;
  hipLaunchKernelGGL(k_parity_to_f32, dim3((unsigned)((n6 + 255) / 256)), dim3(256), 0, s, (f4_t*)y, x, n6, vh);
  return hipGetLastError();
}

hipError_t launch_parity_to_f64(d2_t* y, const void* x, int nrhs, int vh, hipStream_t s) {
  const long long n6 = 6LL * vh * nrhs;
  hipLaunchKernelGGL(k_parity_to_f64, dim3((unsigned)((n6 + 255) / 256)), dim3(256), 0, s, y, (const f4_t*)x, n6, vh);
  return hipGetLastError();
}

}  // namespace ddq
