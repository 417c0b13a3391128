// coarse.hip -- the coarse-grid operator of Sect. 2.3 on several right-hand sides,
//   y(x) = sum over d of A(x, d) v(x + d),
// nine 2N_v x 2N_v complex blocks per coarse site (d = 0 the site's own, d = 1 + 2 mu + s
// the neighbour in direction mu, forward s = 0 or backward s = 1, periodic), FP32
// operands and accumulation, on the matrix cores.
//
// The contraction per block is a complex (2N_v x 2N_v) x (2N_v x nrhs) product: per
// 4-wide slice k of the contraction index and per 16 x 16 output tile, Gauss's three real
// products (the default) or the four of the schoolbook form, with v_mfma_f32_16x16x4_f32, whose operand
// lane l holds A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16] and whose
// accumulator element e of lane l is C[4 (l / 16) + e][l % 16].
//
// Blocks are repacked once (k_coarse_pack) into that operand order, zero-padded to whole
// tiles, two k-slices per 16-byte lane element:
//   packed[x][d][kp][t][lane][4] = (Re, Im) A[16 t + l % 16][8 kp + l / 16]     (slice 2kp)
//                                  (Re, Im) A[16 t + l % 16][8 kp + 4 + l / 16] (slice 2kp+1)
// so a wave reads 1 KB contiguous per load.  A wave of the apply owns one coarse site and
// up to TN tiles of 16 right-hand sides: every block element it loads feeds TN tiles.  Up to
// four such waves (consecutive groups of TN tiles of the same site) form one workgroup, so
// that beyond 16 TN right-hand sides the site's further groups take its blocks from the
// caches while the first wave brings them from memory.
// Two waves per SIMD are asked for (amdgpu_waves_per_eu): the three-product form with 4
// tiles then keeps its 144 accumulators and both operand buffers in the 256 registers
// of a lane (at one wave per SIMD it ran 20% slower).
// Vectors are complex64 [site][row][rhs] (rhs innermost): the 16 lanes of one row read or
// write 128 contiguous bytes.
#include <hip/hip_runtime.h>

#include "coarse_internal.h"

namespace ddq {

namespace {

typedef float f4v __attribute__((ext_vector_type(4)));
typedef float f2v __attribute__((ext_vector_type(2)));

// packed block storage: 4 values per lane element (FP32: 16 bytes; FP16 / BF16: 8 bytes,
// widened to FP32 in registers before the products)
template <typename S>
struct Store4 {
  typedef S v __attribute__((ext_vector_type(4)));
};
template <>
struct Store4<float> {
  typedef f4v v;
};

// FP16 rounds once from the caller's values; BF16 through FP32 (two roundings from FP64)
template <typename S, typename R>
__device__ __forceinline__ S to_store(R r) {
  if constexpr (sizeof(S) == 2 && __is_same(S, __bf16))
    return (S)(float)r;
  else
    return (S)r;
}

template <typename S>
__device__ __forceinline__ f4v widen(typename Store4<S>::v q) {
  if constexpr (sizeof(S) == 4)
    return q;
  else
    return f4v{(float)q[0], (float)q[1], (float)q[2], (float)q[3]};
}

#ifndef DDQ_COARSE_TMAP
#define DDQ_COARSE_TMAP 2
#endif

struct CoarseGeo {
  int cd[4];  // coarse extents
  int n2;     // 2 N_v
  int MT;     // row tiles: ceil(n2 / 16)
  int KP;     // pairs of k-slices: ceil(n2 / 8)
  int vc;     // coarse sites
  int xcd_map;   // order of sites over workgroups w (one site per workgroup column):
                 // 2 (T % 8 == 0): XCD w % 8 takes t-slices [(w % 8) T/8, (w % 8 + 1) T/8), walked
                 //   t fastest, so that every neighbour of a site is a few hundred sites away;
                 // 1 (vc % 8 == 0): XCD w % 8 takes the (w % 8)-th eighth of the sites in order;
                 // 0: site w
};

__device__ __forceinline__ int coarse_nbr(const CoarseGeo& g, int x, int d) {
  if (d == 0) return x;
  const int mu = (d - 1) >> 1;
  int c[4], r = x;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    c[k] = r % g.cd[k];
    r /= g.cd[k];
  }
  c[mu] += ((d - 1) & 1) ? g.cd[mu] - 1 : 1;
  if (c[mu] >= g.cd[mu]) c[mu] -= g.cd[mu];
  return c[0] + g.cd[0] * (c[1] + g.cd[1] * (c[2] + g.cd[2] * c[3]));
}

// one thread per packed lane element; src complex [x][d][i][k] (row-major blocks)
template <typename R, typename S>
__global__ void __launch_bounds__(256) k_coarse_pack(CoarseGeo g, const R* __restrict__ src,
                                                     typename Store4<S>::v* __restrict__ dst, long long n_el) {
  // grid-stride: the grid is capped so that a dispatch stays below 2^32 work-items
  for (long long e = (long long)blockIdx.x * 256 + threadIdx.x; e < n_el; e += (long long)gridDim.x * 256) {
  const int lane = (int)(e & 63);
  long long r = e >> 6;
  const int t = (int)(r % g.MT);
  r /= g.MT;
  const int kp = (int)(r % g.KP);
  const long long xd = r / g.KP;  // x * 9 + d
  const int i = 16 * t + (lane & 15);
  const R* blk = src + xd * 2 * (long long)g.n2 * g.n2;
  S o[4];
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = 8 * kp + 4 * h + (lane >> 4);
    const bool in = i < g.n2 && k < g.n2;
    o[2 * h] = to_store<S>(in ? blk[2 * ((long long)i * g.n2 + k)] : R(0));
    o[2 * h + 1] = to_store<S>(in ? blk[2 * ((long long)i * g.n2 + k) + 1] : R(0));
  }
  dst[e] = typename Store4<S>::v{o[0], o[1], o[2], o[3]};
  // the store reads its data registers after issue; the next iteration rewrites them
  __builtin_amdgcn_sched_barrier(0);
  __builtin_amdgcn_s_waitcnt(0xCF0F);  // expcnt(0)
  __builtin_amdgcn_sched_barrier(0);
  }
}

// operands of one pair of k-slices: the packed block slice and the right-hand sides' rows
template <int MT, int TN>
struct CoarseSlice {
  f4v a[MT];
  float2 b[2][TN];
};

// buffer resource over one coarse site's vector (n2 x nrhs complex64); dword 3 is the
// gfx9 default (32-bit data format, no swizzle)
__device__ __forceinline__ __amdgpu_buffer_rsrc_t site_rsrc(const float2* vn, int bytes) {
  return __builtin_amdgcn_make_buffer_rsrc((void*)vn, (short)0, bytes, 0x00020000);
}

// Rows k >= 2 N_v and columns j >= nrhs read as zero: their offset lies past the
// resource's extent, for which buffer loads return 0.  Every lane issues every load, so
// the loads in flight are counted statically and the products of one slice wait only for
// that slice's own operands.
template <int MT, int TN, typename S>
__device__ __forceinline__ void coarse_load(CoarseSlice<MT, TN>& o, const typename Store4<S>::v* Akp,
                                            __amdgpu_buffer_rsrc_t vr, int kp, int n2, int nrhs, int lk, int j0) {
#pragma unroll
  for (int t = 0; t < MT; ++t) o.a[t] = widen<S>(__builtin_nontemporal_load(Akp + t * 64));
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    const int k = 8 * kp + 4 * h + lk;
#pragma unroll
    for (int n = 0; n < TN; ++n) {
      const int j = j0 + 16 * n;
      const int off = (k < n2 && j < nrhs) ? (k * nrhs + j) * 8 : 0x7ffffff0;
      const f2v t = __builtin_bit_cast(f2v, __builtin_amdgcn_raw_buffer_load_b64(vr, off, 0, 0));
      o.b[h][n] = float2{t.x, t.y};
    }
  }
}

// One step's products.  G3 = 0: four real products per complex one (Yr += Ar Vr - Ai Vi,
// Yi += Ar Vi + Ai Vr) into acc[0] = Yr, acc[1] = Yi.  G3 = 1: Gauss's three real products,
// P += Ar (Vr + Vi), Q += (Ar + Ai) Vi, R += (Ai - Ar) Vr into acc[0..2], with Yr = P - Q and
// Yi = P + R formed once at the end (the sums are rounded to FP32 before the product).
template <int MT, int TN, int G3>
__device__ __forceinline__ void coarse_mma(const CoarseSlice<MT, TN>& c, f4v (&acc)[2 + G3][TN][MT]) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {
    float ar[MT], ai[MT], as[MT], ad[MT];
#pragma unroll
    for (int t = 0; t < MT; ++t) {
      ar[t] = c.a[t][2 * h];
      ai[t] = c.a[t][2 * h + 1];
      as[t] = ar[t] + ai[t];
      ad[t] = ai[t] - ar[t];
    }
#pragma unroll
    for (int n = 0; n < TN; ++n) {
      const float2 b = c.b[h][n];
      const float bs = b.x + b.y;
#pragma unroll
      for (int t = 0; t < MT; ++t) {
        if constexpr (G3) {
          acc[0][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[t], bs, acc[0][n][t], 0, 0, 0);
          acc[1][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(as[t], b.y, acc[1][n][t], 0, 0, 0);
          acc[2][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ad[t], b.x, acc[2][n][t], 0, 0, 0);
        } else {
          acc[0][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[t], b.x, acc[0][n][t], 0, 0, 0);
          acc[0][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(-ai[t], b.y, acc[0][n][t], 0, 0, 0);
          acc[1][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ar[t], b.y, acc[1][n][t], 0, 0, 0);
          acc[1][n][t] = __builtin_amdgcn_mfma_f32_16x16x4f32(ai[t], b.x, acc[1][n][t], 0, 0, 0);
        }
      }
    }
  }
}

// position of the next load in the sequence of (block d, k-slice pair kp), storage order
struct CoarseCursor {
  int q, d, kp;  // linear step, block, slice pair; wraps to the start past the end
  __amdgpu_buffer_rsrc_t vr;
};

template <int MT, int TN, int G3, typename S>
__global__ void __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2))) k_coarse_apply(CoarseGeo g, int nrhs,
                                                                                              const typename Store4<S>::v* __restrict__ A,
                                                     const float2* __restrict__ v, float2* __restrict__ y) {
  const int w = (int)blockIdx.x;
  int x = w;
  if (g.xcd_map == 2) {
    const int tc = g.cd[3] >> 3, q = w >> 3, r = q / tc;
    const int t = (w & 7) * tc + (q - r * tc), xy = g.cd[0] * g.cd[1];
    x = r % xy + xy * (r / xy + g.cd[2] * t);
  } else if (g.xcd_map == 1) {
    x = (w & 7) * (g.vc >> 3) + (w >> 3);
  }
  const int l = (int)threadIdx.x, li = l & 15, lk = l >> 4;
  // the waves of a workgroup share the site and take consecutive groups of TN tiles
  const int grp = (int)(blockIdx.y * blockDim.y + threadIdx.y);
  if (grp * 16 * TN >= nrhs) return;  // a whole wave past the last group
  const int j0 = 16 * TN * grp + li;  // this lane's column in tile 0
  const size_t vstride = (size_t)g.n2 * nrhs;
  const int vbytes = g.n2 * nrhs * 8;
  f4v acc[2 + G3][TN][MT];
#pragma unroll
  for (int q = 0; q < 2 + G3; ++q)
#pragma unroll
    for (int n = 0; n < TN; ++n)
#pragma unroll
      for (int t = 0; t < MT; ++t) acc[q][n][t] = f4v{0.f, 0.f, 0.f, 0.f};
  // two operand buffers in turn: the loads of step s + 1 are in flight during the
  // products of step s; past the last step the cursor re-reads the first (unused)
  const typename Store4<S>::v* Ax = A + (size_t)x * 9 * g.KP * MT * 64 + l;
  const int nsteps = 9 * g.KP;
  CoarseCursor c{0, 0, 0, site_rsrc(v + (size_t)x * vstride, vbytes)};
  auto load_next = [&](CoarseSlice<MT, TN>& o) {
    coarse_load<MT, TN, S>(o, Ax + (size_t)c.q * MT * 64, c.vr, c.kp, g.n2, nrhs, lk, j0);
    if (++c.q == nsteps) c.q = 0;
    if (++c.kp == g.KP) {
      c.kp = 0;
      c.d = c.d == 8 ? 0 : c.d + 1;
      c.vr = site_rsrc(v + (size_t)coarse_nbr(g, x, c.d) * vstride, vbytes);
    }
  };
  CoarseSlice<MT, TN> b0, b1;
  load_next(b0);
  for (int s = 0; s < nsteps; s += 2) {
    load_next(b1);
    coarse_mma<MT, TN, G3>(b0, acc);
    load_next(b0);
    if (s + 1 < nsteps) coarse_mma<MT, TN, G3>(b1, acc);
  }
  float2* yx = y + (size_t)x * vstride;
#pragma unroll
  for (int n = 0; n < TN; ++n) {
    const int j = j0 + 16 * n;
    if (j >= nrhs) continue;
#pragma unroll
    for (int t = 0; t < MT; ++t)
#pragma unroll
      for (int e = 0; e < 4; ++e) {
        const int i = 16 * t + 4 * lk + e;
        if (i >= g.n2) continue;
        if constexpr (G3)
          yx[(size_t)i * nrhs + j] = float2{acc[0][n][t][e] - acc[1][n][t][e], acc[0][n][t][e] + acc[2][n][t][e]};
        else
          yx[(size_t)i * nrhs + j] = float2{acc[0][n][t][e], acc[1][n][t][e]};
      }
  }
}

hipError_t make_geo(const int cd[4], int nv, CoarseGeo& g) {
  if (nv < 1 || nv > 32) return hipErrorInvalidValue;
  long long vc = 1;
  for (int k = 0; k < 4; ++k) {
    if (cd[k] < 1) return hipErrorInvalidValue;
    g.cd[k] = cd[k];
    vc *= cd[k];
  }
  if (vc > (1LL << 25)) return hipErrorInvalidValue;  // grid.x * 64 work-items stays below 2^31
  g.vc = (int)vc;
  g.n2 = 2 * nv;
  g.MT = (g.n2 + 15) / 16;
  g.KP = (g.n2 + 7) / 8;
  g.xcd_map = (g.cd[3] % 8 == 0) ? DDQ_COARSE_TMAP : (g.vc % 8 == 0) ? 1 : 0;
  return hipSuccess;
}

template <int MT, int G3, typename S>
hipError_t launch_mt(const CoarseGeo& g, int nrhs, int tn, const void* A, const float2* v, float2* y, hipStream_t s) {
  const int tiles = (nrhs + 15) / 16;
  const int groups = (tiles + tn - 1) / tn, wpg = groups < 4 ? groups : 4;
  const dim3 grid((unsigned)g.vc, (unsigned)((groups + wpg - 1) / wpg)), block(64, wpg);
  const typename Store4<S>::v* As = (const typename Store4<S>::v*)A;
  switch (tn) {
    case 1: hipLaunchKernelGGL((k_coarse_apply<MT, 1, G3, S>), grid, block, 0, s, g, nrhs, As, v, y); break;
    case 2: hipLaunchKernelGGL((k_coarse_apply<MT, 2, G3, S>), grid, block, 0, s, g, nrhs, As, v, y); break;
    case 3: hipLaunchKernelGGL((k_coarse_apply<MT, 3, G3, S>), grid, block, 0, s, g, nrhs, As, v, y); break;
    default: hipLaunchKernelGGL((k_coarse_apply<MT, 4, G3, S>), grid, block, 0, s, g, nrhs, As, v, y); break;
  }
  return hipGetLastError();
}

template <int G3, typename S>
hipError_t launch_g(const CoarseGeo& g, int nrhs, int tn, const void* A, const float2* v, float2* y, hipStream_t s) {
  switch (g.MT) {
    case 1: return launch_mt<1, G3, S>(g, nrhs, tn, A, v, y, s);
    case 2: return launch_mt<2, G3, S>(g, nrhs, tn, A, v, y, s);
    case 3: return launch_mt<3, G3, S>(g, nrhs, tn, A, v, y, s);
    default: return launch_mt<4, G3, S>(g, nrhs, tn, A, v, y, s);
  }
}

template <typename S>
hipError_t launch_pack(const CoarseGeo& g, int src_f64, const void* src, void* dst, hipStream_t s) {
  const long long n_el = (long long)g.vc * 9 * g.KP * g.MT * 64;
  const long long blocks = (n_el + 255) / 256;
  const dim3 grid((unsigned)(blocks < (1LL << 20) ? blocks : (1LL << 20))), block(256);
  typename Store4<S>::v* d = (typename Store4<S>::v*)dst;
  if (src_f64)
    hipLaunchKernelGGL((k_coarse_pack<double, S>), grid, block, 0, s, g, (const double*)src, d, n_el);
  else
    hipLaunchKernelGGL((k_coarse_pack<float, S>), grid, block, 0, s, g, (const float*)src, d, n_el);
  return hipGetLastError();
}

}  // namespace

long long coarse_packed_bytes(const int cd[4], int nv, int storage) {
  CoarseGeo g;
  if (make_geo(cd, nv, g) != hipSuccess || storage < COARSE_F32 || storage > COARSE_BF16) return -1;
  return (long long)g.vc * 9 * g.KP * g.MT * 64 * (storage == COARSE_F32 ? 16 : 8);
}

hipError_t launch_coarse_pack(const int cd[4], int nv, int storage, int src_f64, const void* src, void* dst,
                              hipStream_t s) {
  CoarseGeo g;
  hipError_t e = make_geo(cd, nv, g);
  if (e != hipSuccess) return e;
  switch (storage) {
    case COARSE_F32: return launch_pack<float>(g, src_f64, src, dst, s);
    case COARSE_F16: return launch_pack<_Float16>(g, src_f64, src, dst, s);
    case COARSE_BF16: return launch_pack<__bf16>(g, src_f64, src, dst, s);
    default: return hipErrorInvalidValue;
  }
}

hipError_t launch_coarse_apply(const int cd[4], int nv, int storage, int nrhs, int rhs_tiles_per_wave, int product,
                               const void* packed, const void* v, void* y, hipStream_t s) {
  CoarseGeo g;
  hipError_t e = make_geo(cd, nv, g);
  if (e != hipSuccess) return e;
  const int tiles = (nrhs + 15) / 16;
  if (nrhs < 1 || (tiles + 3) / 4 > 65535) return hipErrorInvalidValue;
  if (rhs_tiles_per_wave > 4 || product < 0 || product > 2) return hipErrorInvalidValue;
  if (storage < COARSE_F32 || storage > COARSE_BF16) return hipErrorInvalidValue;
  const int g3 = product != 1;  // the default is Gauss's three products
  // default grouping: the fewest groups of at most 4 tiles (3 for the three-product form
  // with 4 row tiles, whose 4-tile kernel spills), balanced (5 tiles: 3 + 2, not 4 + 1)
  const int max_tn = (g3 && g.MT == 4) ? 3 : 4;
  const int groups = (tiles + max_tn - 1) / max_tn;
  int tn = rhs_tiles_per_wave > 0 ? rhs_tiles_per_wave : (tiles + groups - 1) / groups;
  if (tn > tiles) tn = tiles;
  const float2* vv = (const float2*)v;
  float2* yy = (float2*)y;
  switch (storage) {
    case COARSE_F16:
      return g3 ? launch_g<1, _Float16>(g, nrhs, tn, packed, vv, yy, s) : launch_g<0, _Float16>(g, nrhs, tn, packed, vv, yy, s);
    case COARSE_BF16:
      return g3 ? launch_g<1, __bf16>(g, nrhs, tn, packed, vv, yy, s) : launch_g<0, __bf16>(g, nrhs, tn, packed, vv, yy, s);
    default:
      return g3 ? launch_g<1, float>(g, nrhs, tn, packed, vv, yy, s) : launch_g<0, float>(g, nrhs, tn, packed, vv, yy, s);
  }
}

}  // namespace ddq
