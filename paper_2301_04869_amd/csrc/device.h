// Device-side view of one problem: sizes and device pointers, passed by value
// to every kernel.  Per-scenario arrays are scenario-major ([N][len]).
#pragma once

#include <hip/hip_runtime.h>

#include "layout.h"
#include "rkkt.h"

namespace rkkt {

struct DP {
  int nb, nl, ng, nload, ref, gref, nx, nu, m, nz, N;
  int n_ev, off_P, off_Q, off_gx, off_gu, off_h;
  int nnz_gx, nnz_gu, nnz_h, nnz_k, nnz_f;
  int nlev_up, nlev_dn, col_tile, lds;
  double aref, bref;  // reference generator cost, per-unit coefficients
  // network
  const int *line_f, *line_t, *line_loc;
  const double *gs, *bs, *bc;                 // per line: series conductance, susceptance, half charging
  const int *th_src, *v_src, *prow, *qrow, *pg_u, *gnr, *gen_bus;
  const double *ca, *cb, *cc;                 // per generator cost a Pg^2 + b Pg + c (per unit)
  const int *load_of_bus, *grow_bus, *gen_u;  // load index per bus, bus of every g row, u index of every generator's output
  double *pdb, *qdb;                          // [N][nb] bus loads
  // permutation
  const int *perm, *pinv;
  // gathers
  const int *ev_ptr, *ev_src;
  const double *ev_const;
  const int *gx_ptr, *gx_col, *gxc_ptr, *gxc_row, *gxc_pos;
  const int *gu_ptr, *gu_col, *guc_ptr, *guc_row, *guc_pos;
  const int *h_ptr, *h_col, *ht_ptr, *ht_row, *ht_pos, *h0pos;
  const int *k_ptr, *k_col, *k_diag, *k_usplit, *k_row;
  const int *w_ptr, *w_src, *wp_ptr, *wp_a, *wp_b;
  const double *wp_coef, *w_const;
  const int *t_ptr, *t_row, *t_a, *t_b;
  const int *f_ptr, *f_col, *f_diag, *f_tpos, *gx2f;
  const int *lvu_ptr, *lvu_rows, *lvd_ptr, *lvd_rows;
  // cached values and workspace
  double *LV;      // [N][nl][28]
  double *LH;      // [N][nl][10]
  double *EV;      // [N][n_ev]
  double *W;       // [N][nnz_k]
  double *K;       // [N][nnz_k]
  double *LU;      // [N][nnz_f]
  double *invd;    // [N][nx]
  double *part;    // [N][nu][nu] scenario contributions to the reduced matrix
  double *panel;   // global panels when not LDS-resident: [N][ntile][2][nx][col_tile]
  int *imap;       // refactor column maps when not LDS-resident: [N][4][nx]
  double *rhat1;   // [N][nx] internal order
  double *rpart;   // [N][nu]
  int *status;     // [2]: code, scenario
};

// dynamic LDS limits of the kernels for this problem's sizes; called by rkkt_create
hipError_t configure_lu_kernels(const DP& d);
hipError_t configure_dense_kernels(const DP& d);
void launch_copy(const double* a, double* b, long long n, hipStream_t s);

// launchers (k_eval.hip)
void launch_bus_loads(const DP& d, const double* pd, const double* qd, hipStream_t s);
void launch_evaluate(const DP& d, const double* x, const double* u, const double* y,
                     const double* z, double w, double* f, double* gx, double* gu,
                     double* g, double* h, hipStream_t s);
void launch_condense_values(const DP& d, const double* sx, const double* ss, double dw,
                            hipStream_t s);
// (k_lu.hip)
void launch_refactor(const DP& d, hipStream_t s);
void launch_reduce(const DP& d, hipStream_t s);
void launch_step_rhs(const DP& d, const double* r1x, const double* r2, const double* r3,
                     const double* r4, const double* ss, hipStream_t s);
void launch_step_recover(const DP& d, const double* r2, const double* r3, const double* r4,
                         const double* ss, const double* pu, double* px, double* ps,
                         double* py, double* pz, hipStream_t s);
// (k_dense.hip)
void launch_scenario_sum(const DP& d, const double* su, double dw, double* khat, hipStream_t s);
void launch_cholesky(const DP& d, double* a, int* info, hipStream_t s);
void launch_reduced_solve(const DP& d, const double* r1u, const double* chol, double* pu,
                          hipStream_t s);

}  // namespace rkkt
