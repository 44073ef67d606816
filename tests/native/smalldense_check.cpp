// Host check of the small dense eigensolvers used by the recycling steps:
// reads n and a symmetric n x n matrix (row-major) from stdin, prints the
// eigenvalues (ascending) and the eigenvector matrix of the tridiagonal QR
// route, then the same for the Jacobi route.
#include "../../paper_2306_15049_amd/csrc/smalldense.hpp"
#include <cstdio>
#include <vector>
int main()
{
    int n = 0;
    if (scanf("%d", &n) != 1 || n < 0) return 2;
    std::vector<double> S((size_t)n * n);
    for (auto &v : S)
        if (scanf("%lf", &v) != 1) return 2;
    std::vector<double> w, V;
    const bool ok = rsr::sym_eig_tridiag(n, S.data(), w, V);
    printf("%d\n", ok ? 1 : 0);
    for (double x : w) printf("%.17g\n", x);
    for (double x : V) printf("%.17g\n", x);
    rsr::sym_eig_jacobi(n, S.data(), w, V);
    for (double x : w) printf("%.17g\n", x);
    for (double x : V) printf("%.17g\n", x);
    return 0;
}
