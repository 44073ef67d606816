// Host check of the Cholesky QR factor used in the second pass of the
// principal-space orthonormalisation: reads n and a symmetric positive
// definite n x n matrix (row-major) from stdin, prints 1 and T = L^{-T}
// (column-major) or 0 if the factorisation is refused.
#include "../../paper_2306_15049_amd/csrc/smalldense.hpp"
#include <cstdio>
#include <vector>
int main()
{
    int n = 0;
    if (scanf("%d", &n) != 1 || n < 0) return 2;
    std::vector<double> G((size_t)n * n);
    for (auto &v : G)
        if (scanf("%lf", &v) != 1) return 2;
    std::vector<double> T;
    const bool ok = rsr::chol_qr_factor(n, G.data(), T);
    printf("%d\n", ok ? 1 : 0);
    if (ok)
        for (double x : T) printf("%.17g\n", x);
    return 0;
}
