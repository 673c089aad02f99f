// Device state of the interior-point driver and the launchers of its glue
// kernels (k_ipm.hip).  Arrays are scenario-major; x, y in the external order.
#pragma once

#include "device.h"

namespace rkkt {

struct IpmDev {
  const double *xl, *xu, *ul, *uu, *sl, *su;       // boxes, +-inf when absent
  double *x, *u, *s, *y, *z;                       // iterate
  double *zlx, *zux, *zlu, *zuu, *zls, *zus;       // bound multipliers
  double *xt, *ut, *st;                            // trial primal point
  double *f, *gx, *gu, *g, *h;                     // evaluation at the iterate
  double *ft, *gxt, *gut, *gt, *ht;                // evaluation at the trial point
  double *sx, *sgu, *ss;                           // Sigma_x, Sigma_u, Sigma_s
  double *r1x, *r1u, *r2, *r3, *r4;                // residuals with barrier terms
  double *dx, *du, *ds;                            // dual infeasibility with bound multipliers
  double *cu;                                      // [N][nu] scenario u-gradient of the Lagrangian
  double *px, *pu, *ps, *py, *pz;                  // Newton step
  double *pzlx, *pzux, *pzlu, *pzuu, *pzls, *pzus; // bound-multiplier steps
  double *khat, *chol;
  int* info;
  double* scal;                                    // device scalars [32]
};

void ipm_resid(const DP& d, const IpmDev& s, double mu, hipStream_t st);
void ipm_kkt_scalars(const DP& d, const IpmDev& s, double mu, double* out, hipStream_t st);
void ipm_merit(const DP& d, const IpmDev& s, bool trial, double* out, hipStream_t st);
void ipm_step_scalars(const DP& d, const IpmDev& s, double mu, double tau, double* out,
                      hipStream_t st);
void ipm_trial(const DP& d, const IpmDev& s, double alpha, hipStream_t st);
void ipm_accept(const DP& d, const IpmDev& s, double alpha, double alpha_z, double mu, double ks,
                hipStream_t st);
void ipm_init_primal(const DP& d, const IpmDev& s, double k1, double k2, hipStream_t st);
void ipm_init_slack(const DP& d, const IpmDev& s, double k1, double k2, hipStream_t st);
void ipm_grad_max(const DP& d, const IpmDev& s, double* out, hipStream_t st);
void ipm_warm_primal(const DP& d, const IpmDev& s, const double* x0, const double* u0, double k1, double k2,
                     hipStream_t st);
void ipm_warm_duals(const DP& d, const IpmDev& s, const double* y0, const double* z0, double mult, double mu0,
                    hipStream_t st);
void ipm_warm_implied(const DP& d, const IpmDev& s, double mu0, hipStream_t st);

}  // namespace rkkt
