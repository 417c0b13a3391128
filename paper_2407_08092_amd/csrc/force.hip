// force.hip -- derivative of Re(chi^H D_S(U) phi) with respect to the gauge links.
//
// With D_S = A_ee - H_eo A_oo^-1 H_oe and psi_o = A_oo^-1 H_oe phi_e,
// lambda_o = A_oo^-1 (H^H)_oe chi_e (kernel A, plain and dagger), the variation is
//   dL = Re[ chi^H dA_ee phi + lambda^H dA_oo psi - chi^H dH_eo psi - lambda^H dH_oe phi ].
// Every term is Re tr(dU M) for a 3x3 matrix M per link; the gradient in torch's
// convention (dL = Re tr(G^H dU)) is G = M^H, and the su(3) force under
// U -> exp(i e T_a) U is F_a = -Im tr(T_a U M).
//
// Hopping part, link U_mu(y): it enters H once as a forward hop out of y and once
// as a backward hop out of y + mu; for a pair (a on rows, b on columns)
//   a^H (1 - g_mu) dU b(y+mu) = tr(dU sum_s [(1 - g_mu) b(y+mu)]_s a(y)_s^H),
//   a^H (1 + g_mu) dU^H b(y)  = conj-transposed of the same with (1 + g_mu).
// Clover part: per site x and plane (p < q) the insertion
//   W~_pq(x) = (W - W^H) / 8,  W = (i c_sw / 2) sum_s (sigma_pq b)_s a_s^H,
// with (a, b) = (chi, phi) on even and (lambda, psi) on odd sites, gives
//   dL = sum_x sum_pq Re tr(dQ_pq(x) W~_pq(x)),
// and each link sits in 2 plaquettes per plane x 3 planes x 4 corners = 24 leaves.
#include "ddq_internal.h"

namespace ddq {

struct C3 {
  cpx<double> a[3][3];
};

__device__ __forceinline__ C3 c3_zero() {
  C3 m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = {0.0, 0.0};
  return m;
}
__device__ __forceinline__ C3 c3_mul(const C3& A, const C3& B) {
  C3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) {
      cpx<double> s = A.a[i][0] * B.a[0][j];
      cfma(s, A.a[i][1], B.a[1][j]);
      cfma(s, A.a[i][2], B.a[2][j]);
      C.a[i][j] = s;
    }
  return C;
}
__device__ __forceinline__ C3 c3_dag(const C3& A) {
  C3 C;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) C.a[i][j] = conj(A.a[j][i]);
  return C;
}
__device__ __forceinline__ void c3_axpy(C3& Y, double s, const C3& X) {
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) Y.a[i][j] = Y.a[i][j] + s * X.a[i][j];
}

__device__ __forceinline__ long long lexf(const Geo& g, const int c[4]) {
  return c[0] + (long long)g.L[0] * (c[1] + (long long)g.L[1] * (c[2] + (long long)g.L[2] * c[3]));
}
__device__ __forceinline__ void shiftc(const Geo& g, int c[4], int mu, int step) {
  c[mu] += step;
  if (c[mu] < 0) c[mu] += g.L[mu];
  if (c[mu] >= g.L[mu]) c[mu] -= g.L[mu];
}
__device__ __forceinline__ C3 link_at(const Geo& g, const d2_t* U, const int c[4], int mu) {
  const d2_t* u = U + (lexf(g, c) * 4 + mu) * 9;
  C3 m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = {u[3 * i + j].x, u[3 * i + j].y};
  return m;
}

// spinor of site with coordinates c from the parity vectors (even / odd)
__device__ __forceinline__ Spinor<double> spinor_at(const Geo& g, const d2_t* ve, const d2_t* vo,
                                                    const int c[4]) {
  const long long n = lexf(g, c);
  const int par = (c[0] + c[1] + c[2] + c[3]) & 1;
  const d2_t* v = par ? vo : ve;
  const int i = (int)(n >> 1);
  Spinor<double> s;
  for (int sp = 0; sp < 4; ++sp)
    for (int co = 0; co < 3; ++co) {
      d2_t z = v[(size_t)(3 * sp + co) * g.Vh + i];
      s.c[sp][co] = {z.x, z.y};
    }
  return s;
}

// sigma_pq b in the chiral basis: block diagonal, upper spins 0,1 and lower 2,3.
//   sigma_{l t} = diag(s_l, -s_l),  sigma_{jk} = -eps_{jkl} diag(s_l, s_l)
// plane index: 0 (x,y), 1 (x,z), 2 (x,t), 3 (y,z), 4 (y,t), 5 (z,t)
__device__ __forceinline__ void pauli(int l, const cpx<double> u[2], cpx<double> o[2]) {
  if (l == 0) {  // s1
    o[0] = u[1];
    o[1] = u[0];
  } else if (l == 1) {  // s2 = [[0, -i], [i, 0]]
    o[0] = times_minus_i(u[1]);
    o[1] = times_i(u[0]);
  } else {  // s3
    o[0] = u[0];
    o[1] = {-u[1].r, -u[1].i};
  }
}

__device__ __forceinline__ Spinor<double> sigma_mul(int plane, const Spinor<double>& b) {
  // (pauli index l, upper sign, lower sign)
  int l;
  double su, sl;
  switch (plane) {
    case 0: l = 2; su = -1; sl = -1; break;  // sigma_xy = -diag(s3, s3)
    case 1: l = 1; su = 1; sl = 1; break;    // sigma_xz = +diag(s2, s2)
    case 2: l = 0; su = 1; sl = -1; break;   // sigma_xt = diag(s1, -s1)
    case 3: l = 0; su = -1; sl = -1; break;  // sigma_yz = -diag(s1, s1)
    case 4: l = 1; su = 1; sl = -1; break;   // sigma_yt = diag(s2, -s2)
    default: l = 2; su = 1; sl = -1; break;  // sigma_zt = diag(s3, -s3)
  }
  Spinor<double> o;
  for (int c = 0; c < 3; ++c) {
    cpx<double> u[2], r[2];
    u[0] = b.c[0][c];
    u[1] = b.c[1][c];
    pauli(l, u, r);
    o.c[0][c] = su * r[0];
    o.c[1][c] = su * r[1];
    u[0] = b.c[2][c];
    u[1] = b.c[3][c];
    pauli(l, u, r);
    o.c[2][c] = sl * r[0];
    o.c[3][c] = sl * r[1];
  }
  return o;
}

// per site: W~_pq = (W - W^H) / 8 with W = (i c_sw / 2) sum_s (sigma_pq b)_s a_s^H,
// stored [site (lexicographic)][plane 6][3][3]
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1))) k_force_insertions(Geo g, const d2_t* __restrict__ chi_e, const d2_t* __restrict__ lam_o,
                                   const d2_t* __restrict__ phi_e, const d2_t* __restrict__ psi_o, double c_sw,
                                   d2_t* __restrict__ W) {
  const long long n = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= 2LL * g.Vh) return;
  int c[4];
  {
    long long r = n;
    c[0] = (int)(r % g.L[0]);
    r /= g.L[0];
    c[1] = (int)(r % g.L[1]);
    r /= g.L[1];
    c[2] = (int)(r % g.L[2]);
    c[3] = (int)(r / g.L[2]);
  }
  const Spinor<double> a = spinor_at(g, chi_e, lam_o, c);
  const Spinor<double> b = spinor_at(g, phi_e, psi_o, c);
  const double h = 0.5 * c_sw;
  for (int plane = 0; plane < 6; ++plane) {
    const Spinor<double> sb = sigma_mul(plane, b);
    C3 K = c3_zero();
    for (int s = 0; s < 4; ++s)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) cfma(K.a[i][j], sb.c[s][i], conj(a.c[s][j]));
    // W = i h K;  W~ = (W - W^H) / 8
    d2_t* out = W + (n * 6 + plane) * 9;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cpx<double> wij = h * times_i(K.a[i][j]);
        cpx<double> wji = h * times_i(K.a[j][i]);
        d2_t v;
        v.x = 0.125 * (wij.r - wji.r);
        v.y = 0.125 * (wij.i + wji.i);
        out[3 * i + j] = v;
        store_fence();
      }
  }
}

__device__ __forceinline__ C3 insertion_at(const Geo& g, const d2_t* W, const int c[4], int plane) {
  const d2_t* w = W + (lexf(g, c) * 6 + plane) * 9;
  C3 m;
  for (int i = 0; i < 3; ++i)
    for (int j = 0; j < 3; ++j) m.a[i][j] = {w[3 * i + j].x, w[3 * i + j].y};
  return m;
}

__device__ __forceinline__ int plane_of(int p, int q) {  // p < q
  return p == 0 ? q - 1 : (p == 1 ? q + 1 : 5);
}

// M += s * [U2 U3 U4 W0 + W1 U2 U3 U4 + U2 W2 U3 U4 + U2 U3 W3 U4] for the loop
// U1 U2 U3 U4 through the corners c0..c3 (U1 the link itself, leaving c0)
__device__ void add_leaves(C3& M, double s, const C3& U2, const C3& U3, const C3& U4, const C3& W0,
                           const C3& W1, const C3& W2, const C3& W3) {
  const C3 U34 = c3_mul(U3, U4);
  const C3 U234 = c3_mul(U2, U34);
  C3 acc = c3_mul(U234, W0);
  C3 t = c3_mul(W1, U234);
  c3_axpy(acc, 1.0, t);
  t = c3_mul(c3_mul(U2, W2), U34);
  c3_axpy(acc, 1.0, t);
  t = c3_mul(c3_mul(c3_mul(U2, U3), W3), U4);
  c3_axpy(acc, 1.0, t);
  c3_axpy(M, s, acc);
}

// One thread per link U_mu(y).  Outputs G = M^H (torch convention) and/or the
// su(3) projection F_a = -Im tr(T_a U M).
__global__ void __launch_bounds__(128) __attribute__((amdgpu_waves_per_eu(1, 1))) k_force_links(Geo g, const d2_t* __restrict__ U, const d2_t* __restrict__ W,
                                                     const d2_t* __restrict__ chi_e, const d2_t* __restrict__ lam_o,
                                                     const d2_t* __restrict__ phi_e, const d2_t* __restrict__ psi_o,
                                                     d2_t* __restrict__ G, double* __restrict__ F, int accum) {
  const long long tid = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (tid >= 8LL * g.Vh) return;
  const int mu = (int)(tid & 3);
  const long long n = tid >> 2;
  int y[4];
  {
    long long r = n;
    y[0] = (int)(r % g.L[0]);
    r /= g.L[0];
    y[1] = (int)(r % g.L[1]);
    r /= g.L[1];
    y[2] = (int)(r % g.L[2]);
    y[3] = (int)(r / g.L[2]);
  }
  int yp[4] = {y[0], y[1], y[2], y[3]};
  shiftc(g, yp, mu, 1);
  const double bsign = (g.antiperiodic && mu == 3 && y[3] == g.L[3] - 1) ? -1.0 : 1.0;

  C3 M = c3_zero();
  // ---- hopping: forward use out of y, backward use out of y + mu ----
  {
    // a on rows, b on columns: rows of parity(y) use (chi, phi-side) or (lambda, psi-side)
    const Spinor<double> a_y = spinor_at(g, chi_e, lam_o, y);
    const Spinor<double> b_yp = spinor_at(g, phi_e, psi_o, yp);
    const Spinor<double> a_yp = spinor_at(g, chi_e, lam_o, yp);
    const Spinor<double> b_y = spinor_at(g, phi_e, psi_o, y);
    // (1 -+ g_mu) b through the projector identity (h, sg B^H h), h = b_up + sg B b_dn
    Spinor<double> pf, pb;
    zero(pf);
    zero(pb);
    switch (mu) {
      case 0: accumulate<0, double>(pf, project<0, double>(b_yp, -1.0), -1.0);
              accumulate<0, double>(pb, project<0, double>(b_y, 1.0), 1.0); break;
      case 1: accumulate<1, double>(pf, project<1, double>(b_yp, -1.0), -1.0);
              accumulate<1, double>(pb, project<1, double>(b_y, 1.0), 1.0); break;
      case 2: accumulate<2, double>(pf, project<2, double>(b_yp, -1.0), -1.0);
              accumulate<2, double>(pb, project<2, double>(b_y, 1.0), 1.0); break;
      default: accumulate<3, double>(pf, project<3, double>(b_yp, -1.0), -1.0);
               accumulate<3, double>(pb, project<3, double>(b_y, 1.0), 1.0); break;
    }
    // M_f = sum_s pf_s a(y)_s^H ;  M_b = sum_s pb_s a(y+mu)_s^H ;  M += -1/2 s (M_f + M_b^H)
    C3 Mf = c3_zero(), Mb = c3_zero();
    for (int s = 0; s < 4; ++s)
      for (int i = 0; i < 3; ++i)
        for (int j = 0; j < 3; ++j) {
          cfma(Mf.a[i][j], pf.c[s][i], conj(a_y.c[s][j]));
          cfma(Mb.a[i][j], pb.c[s][i], conj(a_yp.c[s][j]));
        }
    c3_axpy(M, -0.5 * bsign, Mf);
    c3_axpy(M, -0.5 * bsign, c3_dag(Mb));
  }
  // ---- clover: 3 planes x 2 plaquettes x 4 corners ----
  for (int nu = 0; nu < 4; ++nu) {
    if (nu == mu) continue;
    const int plane = mu < nu ? plane_of(mu, nu) : plane_of(nu, mu);
    const double o = mu < nu ? 1.0 : -1.0;
    // upper plaquette: y -> y+mu -> y+mu+nu -> y+nu -> y
    {
      int c1[4] = {yp[0], yp[1], yp[2], yp[3]};
      int c2[4] = {yp[0], yp[1], yp[2], yp[3]};
      shiftc(g, c2, nu, 1);
      int c3[4] = {y[0], y[1], y[2], y[3]};
      shiftc(g, c3, nu, 1);
      const C3 U2 = link_at(g, U, c1, nu);
      const C3 U3 = c3_dag(link_at(g, U, c3, mu));
      const C3 U4 = c3_dag(link_at(g, U, y, nu));
      add_leaves(M, o, U2, U3, U4, insertion_at(g, W, y, plane), insertion_at(g, W, c1, plane),
                 insertion_at(g, W, c2, plane), insertion_at(g, W, c3, plane));
    }
    // lower plaquette: y -> y+mu -> y+mu-nu -> y-nu -> y (opposite orientation)
    {
      int c1[4] = {yp[0], yp[1], yp[2], yp[3]};
      int c2[4] = {yp[0], yp[1], yp[2], yp[3]};
      shiftc(g, c2, nu, -1);
      int c3[4] = {y[0], y[1], y[2], y[3]};
      shiftc(g, c3, nu, -1);
      const C3 U2 = c3_dag(link_at(g, U, c2, nu));
      const C3 U3 = c3_dag(link_at(g, U, c3, mu));
      const C3 U4 = link_at(g, U, c3, nu);
      add_leaves(M, -o, U2, U3, U4, insertion_at(g, W, y, plane), insertion_at(g, W, c1, plane),
                 insertion_at(g, W, c2, plane), insertion_at(g, W, c3, plane));
    }
  }
  const long long li = n * 4 + mu;
  if (G) {
    d2_t* out = G + li * 9;
    for (int i = 0; i < 3; ++i)
      for (int j = 0; j < 3; ++j) {
        cpx<double> v = conj(M.a[j][i]);
        d2_t o = out[3 * i + j];
        if (accum) {
          o.x += v.r;
          o.y += v.i;
        } else {
          o.x = v.r;
          o.y = v.i;
        }
        out[3 * i + j] = o;
        store_fence();
      }
  }
  if (F) {
    // UM = U M;  F_a = -Im tr(T_a UM), T_a = lambda_a / 2
    const C3 UM = c3_mul(link_at(g, U, y, mu), M);
    const double r3 = 0.57735026918962576451;  // 1 / sqrt(3)
    double f[8];
    // -Im tr(T_a X), T_a = lambda_a / 2, X = U M, written out per Gell-Mann matrix;
    // for the antisymmetric ones (a = 2, 5, 7) Im(-i X_ji + i X_ij) = Re X_ij - Re X_ji
    f[0] = -0.5 * (UM.a[1][0].i + UM.a[0][1].i);
    f[1] = 0.5 * (UM.a[1][0].r - UM.a[0][1].r);
    f[2] = -0.5 * (UM.a[0][0].i - UM.a[1][1].i);
    f[3] = -0.5 * (UM.a[2][0].i + UM.a[0][2].i);
    f[4] = 0.5 * (UM.a[2][0].r - UM.a[0][2].r);
    f[5] = -0.5 * (UM.a[2][1].i + UM.a[1][2].i);
    f[6] = 0.5 * (UM.a[2][1].r - UM.a[1][2].r);
    f[7] = -0.5 * r3 * (UM.a[0][0].i + UM.a[1][1].i - 2.0 * UM.a[2][2].i);
    double* outf = F + li * 8;
    for (int k = 0; k < 8; ++k) {
      outf[k] = accum ? outf[k] + f[k] : f[k];
      store_fence();
    }
  }
}

hipError_t launch_force(const Geo& g, const d2_t* U, const d2_t* chi_e, const d2_t* lam_o, const d2_t* phi_e,
                        const d2_t* psi_o, double c_sw, d2_t* W, d2_t* G, double* F, int accumulate,
                        hipStream_t s) {
  const long long nsite = 2LL * g.Vh;
  hipLaunchKernelGGL(k_force_insertions, dim3((unsigned)((nsite + 127) / 128)), dim3(128), 0, s, g, chi_e, lam_o,
                     phi_e, psi_o, c_sw, W);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  const long long nlink = 4 * nsite;
  hipLaunchKernelGGL(k_force_links, dim3((unsigned)((nlink + 127) / 128)), dim3(128), 0, s, g, U, W, chi_e, lam_o,
                     phi_e, psi_o, G, F, accumulate);
  return hipGetLastError();
}

}  // namespace ddq
