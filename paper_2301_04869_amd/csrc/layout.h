// Layout of the per-line quantities shared by the symbolic layer (which builds
// gather lists into them) and the kernels (which write them).
#pragma once

#include <hip/hip_runtime.h>

namespace rkkt {

// per (scenario, line): end e in {0: from, 1: to} at offset 14*e holds
// P, Q, dP[4], dQ[4], d|S|^2[4] over the locals (th_f, th_t, v_f, v_t)
constexpr int kLVsize = 28;
constexpr int kLVP = 0, kLVQ = 1, kLVdP = 2, kLVdQ = 6, kLVdS = 10;
// per (scenario, line): upper triangle of the local 4x4 Hessian
constexpr int kLHsize = 10;

__host__ __device__ inline int lh_index(int a, int b) {  // a <= b
  return (a == 0 ? 0 : a == 1 ? 4 : a == 2 ? 7 : 9) + (b - a);
}

}  // namespace rkkt

namespace rkkt {

// Sizes that fix the LDS layouts of the level-scheduled kernels.
struct LdsSizes {
  int nx, nu, nz, nnz_f, nnz_k, nnz_gu, nlu, nld, w;
};

// Local reduction workgroup (one scenario, one tile of w columns):
// doubles lu[nnz_f] invd[nx] kv[nnz_k] guv[nnz_gu] T[nx w] Lx[nx w], then
// ints f_ptr[nx+1] f_diag[nx] f_col[nnz_f] f_tpos[nnz_f] lvu_ptr[nlu+1]
// lvu_rows[nx] lvd_ptr[nld+1] lvd_rows[nx] k_ptr[nz+1] k_usplit[nz]
// k_col[nnz_k] guc_ptr[nu+1] guc_row[nnz_gu].
__host__ __device__ inline long long reduce_lds_doubles(const LdsSizes& z) {
  return (long long)z.nnz_f + z.nx + z.nnz_k + z.nnz_gu + 2LL * z.nx * z.w;
}
__host__ __device__ inline long long solve_meta_ints(const LdsSizes& z) {
  return (long long)(z.nx + 1) + z.nx + 2LL * z.nnz_f + (z.nlu + 1) + z.nx + (z.nld + 1) + z.nx;
}
__host__ __device__ inline long long reduce_lds_ints(const LdsSizes& z) {
  return solve_meta_ints(z) + (z.nz + 1) + z.nz + z.nnz_k + (z.nu + 1) + z.nnz_gu;
}
__host__ __device__ inline long long reduce_lds_bytes(const LdsSizes& z) {
  return 8 * reduce_lds_doubles(z) + 4 * reduce_lds_ints(z);
}
// Refactorisation workgroup: doubles lu[nnz_f] invd[nx] rmax[nx], ints
// f_ptr f_diag f_col lvu_ptr lvu_rows and 4 column maps of nx.
__host__ __device__ inline long long refactor_lds_bytes(const LdsSizes& z) {
  return 8LL * (z.nnz_f + 2LL * z.nx) +
         4LL * ((z.nx + 1) + z.nx + z.nnz_f + (z.nlu + 1) + z.nx + 4LL * z.nx);
}
// Single-column step workgroup: doubles lu invd and three nx vectors, then the
// solve metadata.
__host__ __device__ inline long long step_lds_bytes(const LdsSizes& z) {
  return 8LL * (z.nnz_f + 4LL * z.nx) + 4 * solve_meta_ints(z);
}

}  // namespace rkkt
