// Host check of the one-sided Jacobi SVD used by the principal-space
// stabilisation: reads r, m and an r x m matrix (row-major) from stdin, prints
// the singular values (descending) and the left singular vectors
// (column-major r x r).
#include "../../paper_2306_15049_amd/csrc/smalldense.hpp"
#include <cstdio>
#include <vector>
int main()
{
    int r = 0, m = 0;
    if (scanf("%d %d", &r, &m) != 2 || r < 0 || m < 0) return 2;
    std::vector<double> R((size_t)r * m);
    for (auto &v : R)
        if (scanf("%lf", &v) != 1) return 2;
    std::vector<double> s, U;
    rsr::left_svd_jacobi(r, m, R.data(), s, U);
    for (double x : s) printf("%.17g\n", x);
    for (double x : U) printf("%.17g\n", x);
    return 0;
}
