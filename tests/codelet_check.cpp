// Register DFT codelets against the DFT definition (host build, no device):
// prints the relative error of each size, sign and precision.
#include "dft_codelets.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>

using namespace vloc;

template <int R, int S, typename T>
double check()
{
    double worst = 0;
    for (int trial = 0; trial < 20; ++trial) {
        T xr[R], xi[R];
        double ar[R], ai[R];
        for (int i = 0; i < R; ++i) {
            ar[i] = T(drand48() - 0.5);
            ai[i] = T(drand48() - 0.5);
            xr[i] = T(ar[i]);
            xi[i] = T(ai[i]);
        }
        Dft<R, S, T>::run(xr, xi);
        double err = 0, nrm = 0;
        for (int k = 0; k < R; ++k) {
            long double sr = 0, si = 0;
            for (int n = 0; n < R; ++n) {
                long double a = S * 2.0L * 3.14159265358979323846264338327950288L *
                                (long double)((long)n * k % R) / R;
                sr += ar[n] * cosl(a) - ai[n] * sinl(a);
                si += ar[n] * sinl(a) + ai[n] * cosl(a);
            }
            err += std::pow((double)sr - xr[k], 2) + std::pow((double)si - xi[k], 2);
            nrm += (double)(sr * sr + si * si);
        }
        worst = std::fmax(worst, std::sqrt(err / nrm));
    }
    return worst;
}

#define CASE(R)                                                                                    \
    std::printf("%d %.3e %.3e %.3e %.3e\n", R, check<R, -1, double>(), check<R, 1, double>(),     \
                check<R, -1, float>(), check<R, 1, float>());

int main()
{
    srand48(7);
    CASE(1) CASE(2) CASE(3) CASE(4) CASE(5) CASE(6) CASE(8) CASE(9) CASE(10) CASE(12) CASE(15)
    CASE(16) CASE(18) CASE(20) CASE(24) CASE(25) CASE(27) CASE(30) CASE(32)
    return 0;
}
