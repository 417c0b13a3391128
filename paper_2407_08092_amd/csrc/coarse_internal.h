// coarse_internal.h -- launchers of the coarse-grid operator kernels (coarse.hip).
#pragma once

#include <hip/hip_runtime.h>

namespace ddq {

// storage of the packed blocks
enum { COARSE_F32 = 0, COARSE_F16 = 1, COARSE_BF16 = 2 };

// bytes of the packed block array for coarse extents cd, N_v test vectors and a storage
// (-1 if out of range)
long long coarse_packed_bytes(const int cd[4], int nv, int storage);
// repack complex blocks [site][9][2 N_v][2 N_v] (row-major, complex128 if src_f64 else complex64)
hipError_t launch_coarse_pack(const int cd[4], int nv, int storage, int src_f64, const void* src, void* dst,
                              hipStream_t s);
// y = D_c v on nrhs complex64 right-hand sides, vectors [site][2 N_v][nrhs];
// rhs_tiles_per_wave in 0 (balanced default) .. 4; product 0 (default: three real
// products), 1 (four real products) or 2 (three real products)
hipError_t launch_coarse_apply(const int cd[4], int nv, int storage, int nrhs, int rhs_tiles_per_wave, int product,
                               const void* packed, const void* v, void* y, hipStream_t s);

}  // namespace ddq
