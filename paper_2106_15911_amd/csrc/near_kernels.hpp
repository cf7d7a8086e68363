// Device functions for the nearfield panel integrals (eq. eval_sl_nf_block).
//
// Time integrals are the closed-form second differences of the second
// s-antiderivatives of the heat kernel (G2 for V, K2 for the double layer);
// for time offsets d >= 2 and strong cancellation they are replaced by the
// hat-function integral of the kernel.  Space integrals use the collapsed
// Gauss rule for regular pairs and radial rules for touching pairs
// (identical triangles, common edge, common vertex), whose weights cancel
// the 1/r and 1/r^2 singularities.
#pragma once
#include <hip/hip_runtime.h>

namespace pfmm {

constexpr double kPi = 3.14159265358979323846;
constexpr double kCancel = 1.0e4;
constexpr int kHat = 16;

struct QuadRules {
    double g_reg[16], w_reg[16];
    double g_sing[16], w_sing[16];
    double g_hat[kHat], w_hat[kHat];
    int q_reg, q_sing;
};

__device__ __forceinline__ double G2f(double r, double s, double alpha) {
    if (s <= 0.0) return 0.0;
    const double z = r / (2.0 * sqrt(alpha * s));
    return ((s + r * r / (2.0 * alpha)) * erfc(z) - r * sqrt(s / (kPi * alpha)) * exp(-z * z)) / (4.0 * kPi * alpha * r);
}

__device__ __forceinline__ double K2f(double r, double s, double alpha) {
    if (s <= 0.0) return 0.0;
    const double z = r / (2.0 * sqrt(alpha * s));
    return ((s - r * r / (2.0 * alpha)) * erfc(z) + r * sqrt(s / (kPi * alpha)) * exp(-z * z)) / (4.0 * kPi * r * r * r);
}

__device__ __forceinline__ double Gk(double r, double s, double alpha) {
    return pow(4.0 * kPi * alpha * s, -1.5) * exp(-r * r / (4.0 * alpha * s));
}

// Does the closed-form second difference lose more than ~4 digits?
template <bool K>
__device__ __forceinline__ bool use_hat(double r, int d, double h, double alpha) {
    if (d < 2) return false;
    double big = (d + 1.0) * pow(4.0 * kPi * alpha * d * h, 1.5);
    double lhs;
    if (!K) {
        lhs = kCancel * (4.0 * kPi * alpha) * r * h;
    } else {
        big = 2.0 * d * big;
        lhs = kCancel * (4.0 * kPi) * r * r * r;
    }
    return lhs < big;
}

// int_{(d-1)h}^{(d+1)h} (h - |s - d h|) g(s) ds, g = G (V) or G/(2s) (K).
template <bool K>
__device__ double hat_integral(double r, int d, double h, double alpha, const QuadRules& Q) {
    double sl_sum = 0.0, sr_sum = 0.0;
    for (int i = 0; i < kHat; ++i) {
        const double g = Q.g_hat[i], w = Q.w_hat[i];
        const double sl = (d - 1) * h + h * g;
        const double sr = d * h + h * g;
        double fl = Gk(r, sl, alpha), fr = Gk(r, sr, alpha);
        if (K) { fl = fl / (2.0 * sl); fr = fr / (2.0 * sr); }
        sl_sum += w * g * fl;
        sr_sum += w * (1.0 - g) * fr;
    }
    return (h * h) * (sl_sum + sr_sum);
}

// Accumulate W * timefactor(d) for d = d0 .. min(dmax, d0 + DMAX) at distance
// vector dv into acc[d - d0] (offsets beyond DMAX + 1 take several passes).
template <bool K, int DMAX>
__device__ __forceinline__ void accumulate_point(double acc[DMAX + 1], const double dv[3], const double ny[3], double W,
                                                 int d0, int dmax, double h, double alpha, const QuadRules& Q) {
    const double r = sqrt(dv[0] * dv[0] + dv[1] * dv[1] + dv[2] * dv[2]);
    const double fac = K ? W * (dv[0] * ny[0] + dv[1] * ny[1] + dv[2] * ny[2]) : W;
    auto F = [&](int m) { return m <= 0 ? 0.0 : (K ? K2f(r, m * h, alpha) : G2f(r, m * h, alpha)); };
    double gm1 = F(d0 - 1);                            // F(r, (d-1) h)
    double g0 = F(d0);                                 // F(r, d h)
    double g1 = F(d0 + 1);                             // F(r, (d+1) h)
#pragma unroll
    for (int dd = 0; dd <= DMAX; ++dd) {
        const int d = d0 + dd;
        if (d > dmax) break;
        double v;
        if (d == 0) {
            v = g1;
        } else {
            v = g1 - 2.0 * g0 + gm1;
            if (d >= 2 && use_hat<K>(r, d, h, alpha)) v = hat_integral<K>(r, d, h, alpha, Q);
        }
        acc[dd] += fac * v;
        if (d < dmax) {
            gm1 = g0;
            g0 = g1;
            g1 = F(d + 2);
        }
    }
}

// ---------------------------------------------------------- steps of any length
// Target step [tk0, tk1], source step [tj0, tj1], step-index lag d = k - j.
// The double time integral of G (V) or G / (2 s) (K) is the four-term
// combination of the second s-antiderivative F at the node differences,
//   F(tk1 - tj0) - F(tk1 - tj1) - F(tk0 - tj0) + F(tk0 - tj1),  F(s <= 0) = 0,
// the second difference above when the steps are equal.

// Cancellation test of use_hat with h the longer step and d the lag in units of h.
template <bool K>
__device__ __forceinline__ bool use_overlap(double r, double tk0, double tk1, double tj0, double tj1, double alpha) {
    const double h = fmax(tk1 - tk0, tj1 - tj0);
    const double lag = tk0 - tj0;
    double big = (lag / h + 1.0) * pow(4.0 * kPi * alpha * lag, 1.5);
    double lhs;
    if (!K) {
        lhs = kCancel * (4.0 * kPi * alpha) * r * h;
    } else {
        big = 2.0 * (lag / h) * big;
        lhs = kCancel * (4.0 * kPi) * r * r * r;
    }
    return lhs < big;
}

// int phi(s) g(s) ds over s in [tk0 - tj1, tk1 - tj0], phi(s) the length of
// the overlap of the target step with the source step moved by s: it rises
// over the shorter step length, stays flat over the difference of the two
// lengths and falls over the shorter length again (the hat of hat_integral
// for equal steps); Gauss-Legendre on each piece.
template <bool K>
__device__ double overlap_integral(double r, double tk0, double tk1, double tj0, double tj1, double alpha,
                                   const QuadRules& Q) {
    const double hk = tk1 - tk0, hj = tj1 - tj0;
    const double hm = fmin(hk, hj), flat = fabs(hk - hj);
    const double a = tk0 - tj1, b = a + hm, c = b + flat;
    auto g = [&](double s) { const double v = Gk(r, s, alpha); return K ? v / (2.0 * s) : v; };
    double rise = 0.0, mid = 0.0, fall = 0.0;
    for (int i = 0; i < kHat; ++i) {
        const double x = Q.g_hat[i], w = Q.w_hat[i];
        rise += w * x * g(a + hm * x);
        fall += w * (1.0 - x) * g(c + hm * x);
        if (flat > 0.0) mid += w * g(b + flat * x);
    }
    return hm * hm * (rise + fall) + flat * hm * mid;
}

template <bool K>
__device__ __forceinline__ double time_factor_pair(double r, double tk0, double tk1, double tj0, double tj1, int d,
                                                   double alpha, const QuadRules& Q) {
    if (d >= 2 && use_overlap<K>(r, tk0, tk1, tj0, tj1, alpha)) return overlap_integral<K>(r, tk0, tk1, tj0, tj1, alpha, Q);
    auto F = [&](double s) { return K ? K2f(r, s, alpha) : G2f(r, s, alpha); };
    return F(tk1 - tj0) - F(tk1 - tj1) - F(tk0 - tj0) + F(tk0 - tj1);
}

}  // namespace pfmm
