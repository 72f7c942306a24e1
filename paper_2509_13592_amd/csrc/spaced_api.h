// Entry points of plans on a zero-padded embedding (spaced.cpp), routed to from the C ABI
// when a plan was made by bccb_plan_spaced.  Arguments as the corresponding ABI calls; grids
// are the caller's A1 x A2 grids.
#pragma once

#include "plan_internal.h"

namespace bccb {

int spaced_adjoint(bccb_plan_s* p, const float2* y, float2* b);
int spaced_adjoint_maxabs(bccb_plan_s* p, const float2* y, double* maxabs);
int spaced_gram_apply(bccb_plan_s* p, const float2* x, float2* gx);
int spaced_prox_grad(bccb_plan_s* p, int mode, const float2* y, float tau, int iters, const float2* c0, float2* out);
int spaced_admm(bccb_plan_s* p, const float2* y, float tau, float rho, int iters, float2* zo, float2* co);
int spaced_objective_kkt(bccb_plan_s* p, const float2* y, float tau, const float2* c, double* objective,
                         double* r_kkt, double* max_e_over_tau);

}  // namespace bccb
