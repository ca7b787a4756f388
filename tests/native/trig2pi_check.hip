// Host-side accuracy check of wos::sincos2pi (the FP64 step direction) against long-double sin/cos.
// Usage: trig2pi_check N  -> prints "max_abs_err_sin max_abs_err_cos max_ulp_sin max_ulp_cos"
#include <cmath>
#include <cstdio>
#include <cstdlib>

#include "../../paper_2409_03686_amd/csrc/wos_device.hpp"

static double ulps(double got, long double ref)
{
    const long double a = fabsl(ref);
    if (a < 0.1L) return 0.0;  // ulps only where the value is not near a zero crossing
    int e;
    frexpl(a, &e);
    const long double ulp = ldexpl(1.0L, e - 53);
    return static_cast<double>(fabsl(static_cast<long double>(got) - ref) / ulp);
}

int main(int argc, char **argv)
{
    const long n = argc > 1 ? atol(argv[1]) : 1000000;
    const long double two_pi = 6.283185307179586476925286766559005768L;
    double es = 0, ec = 0, us = 0, uc = 0;
    auto check = [&](double u) {
        double s, c;
        wos::sincos2pi(u, &s, &c);
        const long double th = two_pi * static_cast<long double>(u);
        const long double rs = sinl(th), rc = cosl(th);
        es = fmax(es, static_cast<double>(fabsl(s - rs)));
        ec = fmax(ec, static_cast<double>(fabsl(c - rc)));
        us = fmax(us, ulps(s, rs));
        uc = fmax(uc, ulps(c, rc));
    };
    for (long i = 0; i < n; ++i) check((static_cast<double>(i) + 0.5) / static_cast<double>(n));
    // quarter-turn boundaries and the ends of the uniform's range
    const double edges[] = {0x1.0p-54, 0.125, 0.25, 0.375, 0.5, 0.625, 0.75, 0.875, 1.0 - 0x1.0p-54, 1.0};
    for (double u : edges) {
        check(u);
        check(nextafter(u, 0.0));
        check(nextafter(u, 2.0));
    }
    printf("%.3e %.3e %.3f %.3f\n", es, ec, us, uc);
    return 0;
}
