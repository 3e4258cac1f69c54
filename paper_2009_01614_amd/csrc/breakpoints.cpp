// iSAX region edges: standard-normal quantiles Phi^-1(j / 2^c), j = 1..2^c-1.
//
// The paper cuts the value axis into regions with one bit-string symbol each
// (Sec. II, iSAX Representation) without printing the edges; we use the
// equiprobable cuts of N(0, 1), the usual choice for z-normalised series.
// The quantile function is Wichura's algorithm AS 241 (PPND16, Applied
// Statistics 37(3), 1988): rational approximations in three ranges with
// relative accuracy about 1e-16, evaluated in FP64 and then rounded once to
// the nearest FP32.
#include <cmath>
#include <vector>

#include "internal.h"

namespace isax {
namespace {

double poly(const double* c, int n, double x) {  // c[0] + c[1] x + ... + c[n-1] x^(n-1)
    double r = c[n - 1];
    for (int i = n - 2; i >= 0; --i) r = r * x + c[i];
    return r;
}

double ppnd16(double p) {
    static const double a[8] = {3.3871328727963666080e0, 1.3314166789178437745e+2, 1.9715909503065514427e+3,
                                1.3731693765509461125e+4, 4.5921953931549871457e+4, 6.7265770927008700853e+4,
                                3.3430575583588128105e+4, 2.5090809287301226727e+3};
    static const double b[8] = {1.0, 4.2313330701600911252e+1, 6.8718700749205790830e+2,
                                5.3941960214247511077e+3, 2.1213794301586595867e+4, 3.9307895800092710610e+4,
                                2.8729085735721942674e+4, 5.2264952788528545610e+3};
    static const double c[8] = {1.42343711074968357734e0, 4.63033784615654529590e0, 5.76949722146069140550e0,
                                3.64784832476320460504e0, 1.27045825245236838258e0, 2.41780725177450611770e-1,
                                2.27238449892691845833e-2, 7.74545014278341407640e-4};
    static const double d[8] = {1.0, 2.05319162663775882187e0, 1.67638483018380384940e0,
                                6.89767334985100004550e-1, 1.48103976427480074590e-1, 1.51986665636164571966e-2,
                                5.47593808499534494600e-4, 1.05075007164441684324e-9};
    static const double e[8] = {6.65790464350110377720e0, 5.46378491116411436990e0, 1.78482653991729133580e0,
                                2.96560571828504891230e-1, 2.65321895265761230930e-2, 1.24266094738807843860e-3,
                                2.71155556874348757815e-5, 2.01033439929228813265e-7};
    static const double f[8] = {1.0, 5.99832206555887937690e-1, 1.36929880922735805310e-1,
                                1.48753612908506148525e-2, 7.86869131145613259100e-4, 1.84631831751005468180e-5,
                                1.42151175831644588870e-7, 2.04426310338993978564e-15};
    const double q = p - 0.5;
    if (std::fabs(q) <= 0.425) {
        const double r = 0.180625 - q * q;
        return q * poly(a, 8, r) / poly(b, 8, r);
    }
    double r = q < 0 ? p : 1.0 - p;
    r = std::sqrt(-std::log(r));
    double v;
    if (r <= 5.0) {
        r -= 1.6;
        v = poly(c, 8, r) / poly(d, 8, r);
    } else {
        r -= 5.0;
        v = poly(e, 8, r) / poly(f, 8, r);
    }
    return q < 0 ? -v : v;
}

}  // namespace

std::vector<float> breakpoints_f32(int card_bits) {
    const int ns = 1 << card_bits;
    std::vector<float> out(ns - 1);
    for (int j = 1; j < ns; ++j) out[j - 1] = (float)ppnd16((double)j / ns);
    return out;
}

}  // namespace isax
