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
  int nx, nu, nz, nnz_f, nnz_k, nnz_gu;
  int nnz_l;  // entries of every level-sliced schedule (at most the strict lower count)
  int nlu, nph_u, nph_d, n_upd, w, variant, spw;
  int nph_ru, nph_rd;  // phases of the reduction's schedules
  int upd_lds;  // refactorisation update targets staged in LDS (else read from global)
  int chain_t;  // rows of the chain (its values occupy chain_t^2 doubles in the reduction)
  int nnz_h, m;
};

constexpr int kRedThreads = 1024;  // reduction workgroup
constexpr int kChainMax = 32;      // longest chain of single-row levels solved in registers
constexpr int kGroupLds = 64;      // threads per scenario in the LDS-mode refactor / step
constexpr int kKzItems = 2;        // K-row items per thread held in registers by the LDS-mode reduction
constexpr int kSpSlab = 16;        // stacked rows per slab of the stacked product (chunks are whole slabs)

__host__ __device__ inline int red_slots(const LdsSizes& z) { return kRedThreads / z.w; }

// Local reduction workgroup (one scenario, one tile of w columns): doubles
// lu[nnz_f] invd[nx] kv[nnz_k] guv[nnz_gu] T[nx w] (adjoint variant also
// Lx[nx w]); then packed entries of both solve schedules (2 words each),
// their pointer tables, k_ptr[nz+1] k_usplit[nz] k_col[nnz_k] guc_ptr[nu+1]
// guc_row[nnz_gu].
__host__ __device__ inline long long reduce_lds_doubles(const LdsSizes& z) {
  return (long long)z.nnz_f + z.nx + z.nnz_k + z.nnz_gu + (z.variant == 2 ? 1LL : 2LL) * z.nx * z.w;
}
__host__ __device__ inline long long reduce_lds_ints(const LdsSizes& z) {
  const long long S = red_slots(z);
  return 4LL * z.nnz_l + (z.nph_ru * S + 1) + (z.nph_rd * S + 1) + (z.nz + 1) + z.nz + z.nnz_k +
         (z.nu + 1) + z.nnz_gu + 2;  // + padding to whole 8-byte units
}
// With 64-column tiles the schedule is read from global memory (scalar
// loads); the doubles and the K pattern (k_ptr k_usplit k_col) are staged.
// Both layouts end with the chain block's values (chain_t^2 doubles).
__host__ __device__ inline long long reduce_lds_bytes(const LdsSizes& z) {
  const long long ints = z.w == 64 ? (z.nz + 1) + z.nz + z.nnz_k : reduce_lds_ints(z);
  return 8 * reduce_lds_doubles(z) + 8 * ((ints + 1) / 2) + 8LL * z.chain_t * z.chain_t;
}
// Refactorisation workgroup (spw scenarios, one wavefront each): per scenario
// doubles lu[nnz_f] invd[nx] rmax[nx]; shared packed items (2 words each),
// their pointer table, lvu_ptr lvu_rows f_diag f_ptr, and the update targets
// when upd_lds.
__host__ __device__ inline long long refactor_lds_bytes(const LdsSizes& z) {
  return 8LL * z.spw * (z.nnz_f + 2LL * z.nx) +
         4LL * (2LL * z.nnz_l + (z.nph_u * (long long)kGroupLds + 1) + (z.nlu + 1) + z.nx + z.nx +
                (z.nx + 1) + (z.upd_lds ? (long long)z.n_upd : 0LL) + 2);
}
// Single-column step workgroup (one scenario): doubles lu[nnz_f] invd[nx]
// K[nnz_k] H[nnz_h] G_u[nnz_gu] ra[nx] r3[nx] r2[m] r4[m] ss[m] w[m] v0 v1
// v2 [nx each] pu[nu]; then packed entries of both solve schedules, their
// pointer tables and per-phase largest slot counts.
__host__ __device__ inline long long step_lds_bytes(const LdsSizes& z) {
  return 8LL * ((long long)z.nnz_f + z.nx + z.nnz_k + z.nnz_h + z.nnz_gu + 5LL * z.nx + 4LL * z.m + z.nu) +
         4LL * (4LL * z.nnz_l + (z.nph_u * (long long)kGroupLds + 1) + (z.nph_d * (long long)kGroupLds + 1) +
                z.nph_u + z.nph_d + 2);
}

// step kernels of the stacked variant: lu[nnz_f] invd[nx] v0[nx] v1[nx]
// vu[nu] red[threads + nu] (doubles), then the step schedule blob
__host__ __device__ inline long long step2_lds_bytes(const LdsSizes& z, int threads) {
  return 8LL * ((long long)z.nnz_f + 3LL * z.nx + 2LL * z.nu + threads) +
         4LL * (4LL * z.nnz_l + (z.nph_u * (long long)kGroupLds + 1) + (z.nph_d * (long long)kGroupLds + 1) +
                z.nph_u + z.nph_d + 2);
}

}  // namespace rkkt
