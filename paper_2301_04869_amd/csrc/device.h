// Device-side view of one problem: sizes and device pointers, passed by value
// to every kernel.  Per-scenario arrays are scenario-major ([N][len]).
#pragma once

#include <hip/hip_runtime.h>

#include <utility>
#include <vector>

#include "layout.h"
#include "rkkt.h"

namespace rkkt {

struct DP {
  int nb, nl, ng, nload, ref, gref, nx, nu, m, nz, N;
  int n_ev, off_P, off_Q, off_gx, off_gu, off_h;
  int nnz_gx, nnz_gu, nnz_h, nnz_k, nnz_f, nnz_l;
  int nlev_up, nlev_dn, col_tile;
  int lds_red, lds_grp;   // reduction / refactorisation data in LDS
  int lds_stp;            // step data in LDS
  int spw;                // scenarios per workgroup of the LDS refactor and step
  int upd_lds;            // LDS refactor stages its update targets
  int variant;            // 1 adjoint solves, 2 stacked product
  int nu_pad, nchunk;     // stacked panels: row pitch, contraction chunks
  double aref, bref;  // reference generator cost, per-unit coefficients
  // network
  const int *line_f, *line_t, *line_loc;
  const double *gs, *bs, *bc;                 // per line: series conductance, susceptance, half charging
  const int *th_src, *v_src, *prow, *qrow, *pg_u, *gnr, *gen_bus;
  const double *ca, *cb, *cc;                 // per generator cost a Pg^2 + b Pg + c (per unit)
  const int *load_of_bus, *grow_bus, *gen_u;  // load index per bus, bus of every g row, u index of every generator's output
  double *pdb, *qdb;                          // [N][nb] bus loads
  double *lstat;                              // [N][nl] line admittance factor (1 in service, 0 tripped)
  // permutation
  const int *perm, *pinv;
  // gathers
  const int *ev_ptr, *ev_src;
  const double *ev_const;
  const int *gx_ptr, *gx_col, *gx_row, *gxc_ptr, *gxc_row, *gxc_pos;
  const int *gu_ptr, *gu_col, *guc_ptr, *guc_row, *guc_pos;
  const int *h_ptr, *h_col, *ht_ptr, *ht_row, *ht_pos, *h0pos;
  const int *k_ptr, *k_col, *k_diag, *k_usplit, *k_row;
  const int* kz_items;  // K-row pieces, four ints each (see Sym::kz_items)
  int n_kz, kz_rounds;
  // condensed values with a scenario's sigma_s, H values and triplets in LDS:
  // cv_split workgroups per scenario (0: one thread per value, no LDS), at
  // most cv_nt triplets per workgroup
  int cv_split, cv_nt;
  const int *w_ptr, *w_src, *wp_ptr, *wp_a, *wp_b;
  const double *wp_coef, *w_const;
  const int *t_ptr, *t_row, *t_a, *t_b;
  const int *f_ptr, *f_col, *f_diag, *f_tpos, *gx2f;
  const int *lvu_ptr, *lvu_rows, *lvd_ptr, *lvd_rows;
  // level-sliced schedules: pointer tables and entries (uint2 packed 16-bit
  // pairs when the kernel stages them in LDS, int4 otherwise)
  const int *ru_ptr, *rd_ptr, *su_ptr, *sd_ptr, *fa_ptr;
  const void *ru_ent, *rd_ent, *su_ent, *sd_ent, *fa_ent;
  int nph_u, nph_d, n_upd;  // phases of the step and refactorisation schedules
  int nph_ru, nph_rd;       // phases of the reduction's schedules (ru_*, rd_*)
  int n_sent;             // entries of every schedule (pairs outside the chain)
  int fac_npiv;           // levels whose pivots the refactorisation's phases take
  int chain_t, chain_c0;  // chain rows chain_c0 .. nx - 1
  const int* chain_pos;   // [chain_t][chain_t] filled-pattern positions, -1 absent
  const int* upd_dst;
  int lu_stride;          // nnz_f + nx
  // LDS images of the shared index data of the reduction, the step and the
  // refactorisation, laid out exactly as the kernels' LDS integer regions
  const unsigned *blob_red, *blob_stp, *blob_fac;
  int blob_red_words, blob_stp_words, blob_fac_words;
  // cached values and workspace
  double *LV;      // [N][nl][28]
  double *LH;      // [N][nl][10]
  double *EV;      // [N][n_ev]
  double *W;       // [N][nnz_k]
  double *K;       // [N][nnz_k]
  double *LU;      // [N][lu_stride]: factor values (nnz_f) then 1/u_ii (nx)
  double *part;    // [N][nu][nu] scenario contributions to the reduced matrix
  double *panel;   // global panels when not LDS-resident: [N][ntile][2][nx][col_tile]
  double *Zst;     // stacked product: [N][nz][nu_pad] Z = [-G_x^-1 G_u ; I]
  double *KZst;    // stacked product: [N][nz][nu_pad] K Z
  double *gpart;   // stacked product: [nchunk][nu][nu] lower-triangle partial sums
  double *rhat1;   // [N][nx] internal order
  double *wbuf;    // [N][m] step work vector (global-memory step kernels)
  double *rpart;   // [N][nu]
  double *qbuf;    // [N][nx] internal order: G_x^-1 r3 of the last step right-hand side
  int *status;     // [2]: code, scenario
};

// Copy of n 8-byte units (doubles, or pairs of 32-bit words) from global
// memory into LDS by the threads (start, start + stride, ...): every thread
// issues kStageBatch loads before its first store, so its global round trips
// overlap.  Source and destination are 8-byte aligned.
constexpr int kStageBatch = 16;

template <typename T>
__device__ __forceinline__ void stage_copy(T* __restrict__ dst, const T* __restrict__ src, long long n,
                                           int start, int stride) {
  for (long long i0 = start; i0 < n; i0 += (long long)kStageBatch * stride) {
    T v[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const long long i = i0 + (long long)u * stride;
      if (i < n) v[u] = src[i];
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const long long i = i0 + (long long)u * stride;
      if (i < n) dst[i] = v[u];
    }
  }
}

// the same for an array of 32-bit words padded to an even count
__device__ __forceinline__ void stage_words(void* dst, const void* src, int words, int start, int stride) {
  stage_copy(static_cast<uint2*>(dst), static_cast<const uint2*>(src), (words + 1) / 2, start, stride);
}

// value of v in lane `lane` (wave-uniform) of the calling wavefront
__device__ __forceinline__ double readlane_d(double v, int lane) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, lane);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), lane);
  return __longlong_as_double(((long long)hi << 32) | (unsigned)lo);
}

// value of v in lane Q of the caller's row of 16 lanes (DPP row_newbcast)
template <int Q>
__device__ __forceinline__ double row_bcast(double v) {
  return __builtin_amdgcn_mov_dpp(v, 0x150 + Q, 0xf, 0xf, false);
}

// dst[i * ldd + j] = src[i * lds + j] for i < rows, j < cols, kStageBatch
// loads in flight per thread (dst in LDS)
template <typename T>
__device__ __forceinline__ void copy2d_overlapped(T* dst, int ldd, const T* __restrict__ src, long long lds,
                                                  int rows, int cols, int start, int stride) {
  const int total = rows * cols;
  for (int t0 = start; t0 < total; t0 += kStageBatch * stride) {
    T v[kStageBatch];
    int o[kStageBatch];
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u) {
      const int t = t0 + u * stride;
      o[u] = -1;
      if (t < total) {
        const int i = t / cols, j = t - i * cols;
        v[u] = src[(long long)i * lds + j];
        o[u] = i * ldd + j;
      }
    }
#pragma unroll
    for (int u = 0; u < kStageBatch; ++u)
      if (o[u] >= 0) dst[o[u]] = v[u];
  }
}

// orders the LDS accesses of one wavefront: what its lanes wrote before is
// seen by its lanes after.  A wavefront's LDS operations execute in issue
// order, so this is a compiler barrier only (wavefront-scope fences emit no
// wait): loads issued earlier for later use stay in flight across it.
__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// dynamic LDS limits of the kernels for this problem's sizes; called by rkkt_create
hipError_t configure_lu_kernels(const DP& d);
hipError_t configure_dense_kernels(const DP& d);
void launch_copy(const double* a, double* b, long long n, hipStream_t s);

// launchers (k_eval.hip)
void launch_bus_loads(const DP& d, const double* pd, const double* qd, hipStream_t s);
void launch_line_status(const DP& d, const double* status, hipStream_t s);
void launch_evaluate(const DP& d, const double* x, const double* u, const double* y,
                     const double* z, double w, double* f, double* gx, double* gu,
                     double* g, double* h, hipStream_t s);
void launch_condense_values(const DP& d, const double* sx, const double* ss, double dw,
                            hipStream_t s);
// dynamic LDS limit of the fused line / gather kernel (never lowered)
hipError_t configure_eval_kernels(const DP& d);
// the two halves of launch_evaluate: line values and EV (all that the
// refactorisation needs), then g, h, f, its gradients and W
void launch_evaluate_values(const DP& d, const double* x, const double* u, hipStream_t s);
void launch_evaluate_rest(const DP& d, const double* x, const double* u, const double* y,
                          const double* z, double w, double* f, double* gx, double* gu, double* g,
                          double* h, hipStream_t s);
// (k_lu.hip)
void launch_refactor(const DP& d, hipStream_t s);
void launch_identity_rows(const DP& d, hipStream_t s);
void launch_reduce(const DP& d, hipStream_t s);
void launch_step_rhs(const DP& d, const double* r1x, const double* r2, const double* r3,
                     const double* r4, const double* ss, hipStream_t s);
void launch_step_recover(const DP& d, const double* r2, const double* r3, const double* r4,
                         const double* ss, const double* pu, double* px, double* ps,
                         double* py, double* pz, hipStream_t s);
// (k_dense.hip)
void launch_scenario_sum(const DP& d, const double* su, double dw, double* khat, hipStream_t s);
void launch_stacked_product(const DP& d, hipStream_t s);
void launch_cholesky(const DP& d, double* a, int* info, hipStream_t s);
// factor of src into dst (src is left as it is)
void launch_cholesky_from(const DP& d, const double* src, double* dst, int* info, hipStream_t s);
void launch_reduced_solve(const DP& d, const double* r1u, const double* chol, double* pu,
                          hipStream_t s);

// ---- several independent instances, one launch per kernel configuration
// (rkkt_multi_*).  A Launch is one kernel launch of an instance's pass as its
// single-instance launcher issues it: kernel, template variant, grid gx x gy,
// block threads, dynamic LDS bytes, and for the blocked Cholesky the panel's
// first column jb.  key orders the launches of a pass (stage * 4096 + place
// in the stage), so launches of equal key, kernel, variant and threads from
// several instances become one launch whose blocks map back through MultiBlk.
struct Launch {
  int key, kernel, variant, gx, gy, threads, jb;
  long long lds;
};
struct MultiBlk {
  int inst, bx, by, gx;  // block (bx, by) of instance inst's own grid of width gx
};
enum : int {
  kKLineEvalGather = 1, kKLineEval, kKGatherEv, kKAssemble, kKLineHess, kKWGather, kKCondense,
  kKRefactor, kKReduce64, kKReduce, kKStepRhs2, kKStepRhs, kKStepRec2, kKStepRec,
  kKStacked, kKSymSum, kKCholSmall, kKCopyChol, kKSetInfo, kKCholDiag, kKCholTrsm, kKCholUpdate,
  kKRSolveBlk, kKRSolve, kKCondenseLds
};
enum : int {
  kStEvalValues = 0, kStEvalRest, kStCondense, kStRefactor, kStReduce, kStStepRhs, kStStacked,
  kStSum, kStFactor, kStRSolve, kStRecover
};
// Launches of one pass of instance d (rkkt_iterate on one stream), by stage.
void launches_eval(const DP& d, std::vector<Launch>& out);        // values, rest, condensed values
void launches_lu(const DP& d, std::vector<Launch>& out);          // refactor, reduce, step kernels
void launches_dense(const DP& d, std::vector<Launch>& out);       // product, sum, Cholesky, solve
// One multi-instance launch of l's kernel over nblk blocks (or, with
// prepare, only the dynamic-LDS limit of that kernel); *handled is false when
// the kernel is not in this file.
hipError_t multi_eval(const Launch& l, unsigned nblk, long long lds, const DP* dps, const rkkt_iteration* its,
                      const MultiBlk* blk, hipStream_t s, bool prepare, bool* handled);
hipError_t multi_lu(const Launch& l, unsigned nblk, long long lds, const DP* dps, const rkkt_iteration* its,
                    const MultiBlk* blk, hipStream_t s, bool prepare, bool* handled);
hipError_t multi_dense(const Launch& l, unsigned nblk, long long lds, const DP* dps, const rkkt_iteration* its,
                       const MultiBlk* blk, hipStream_t s, bool prepare, bool* handled);

}  // namespace rkkt
