// Launchers of the outer-iteration kernels (edge weights and L-curve sums of
// Section 2.1, the right-hand side of the correction equation of Section 5.2),
// defined in kernels.hip.
#pragma once
#include "internal.hpp"

namespace rsr {

// edge weights of Sec. 2.1 in place; part: device scratch of edge_rule_parts() doubles
int edge_rule_parts();
hipError_t launch_edge_rule(const double *x, double *wh, double *wv, int ny, int nx, double p, double *part,
                            hipStream_t s);
// L-curve sums of m systems; part: device scratch of 2 * m * lcurve_parts(n) doubles
int lcurve_parts(long n);
hipError_t launch_lcurve(const InstDev *inst_dev, int ii, long n, int m, const double *X, long ld_x,
                         const double *d, double *part, hipStream_t s);

// out = gamma (E_k - E_{k-1}) x from the current and the previous weight planes
hipError_t launch_weight_delta(const double *x, const double *wh, const double *wv, const double *wh0,
                               const double *wv0, double gamma, int ny, int nx, double *out, hipStream_t s);

}  // namespace rsr
