// Encoding by the inverse canonical embedding (paper: Methods, Encode / Decode), FP64 on the host.
//
// Slot j is the evaluation at zeta^(e_j), e_j = 5^j mod 2N, zeta = exp(i pi / N); the conjugate slot
// is at -e_j.  With v_e the slot value at odd exponent e and e = 2k + 1:
//   m_i = (1/N) sum_e v_e zeta^(-i e) = zeta^(-i) * (1/N) sum_k v_{2k+1} omega^(-i k),  omega = zeta^2,
// a length-N complex DFT; decode is the forward transform v_{2k+1} = sum_i (m_i zeta^i) omega^(i k).
#include <cmath>
#include <complex>
#include <map>
#include <mutex>

#include "ckks_internal.h"

namespace gck {

using cd = std::complex<double>;

// twiddles of one stage of the transform, w_j = exp(i ang j) with ang = sign 2 pi / len, made once per
// (len, sign) and shared by every thread afterwards (the values are those the butterflies computed inline)
static const std::vector<cd> &stage_twiddles(size_t len, int sign) {
    static std::mutex mu;
    static std::map<std::pair<size_t, int>, std::vector<cd>> cache;
    std::lock_guard<std::mutex> lk(mu);
    auto &w = cache[{len, sign}];
    if (w.empty()) {
        const double ang = sign * 2.0 * M_PI / (double)len;
        w.resize(len / 2);
        for (size_t j = 0; j < len / 2; ++j) w[j] = cd(std::cos(ang * (double)j), std::sin(ang * (double)j));
    }
    return w;
}

// in-place radix-2 DFT: X_k = sum_i x_i exp(sign * 2 pi i ik / n)
static void fft(std::vector<cd> &a, int sign) {
    const size_t n = a.size();
    for (size_t i = 1, j = 0; i < n; ++i) {
        size_t bit = n >> 1;
        for (; j & bit; bit >>= 1) j ^= bit;
        j ^= bit;
        if (i < j) std::swap(a[i], a[j]);
    }
    for (size_t len = 2; len <= n; len <<= 1) {
        const std::vector<cd> &w = stage_twiddles(len, sign);
        for (size_t s = 0; s < n; s += len) {
            for (size_t j = 0; j < len / 2; ++j) {
                cd u = a[s + j], v = a[s + j + len / 2] * w[j];
                a[s + j] = u + v;
                a[s + j + len / 2] = u - v;
            }
        }
    }
}

static std::vector<u64> slot_exponents(int n) {
    std::vector<u64> e(n / 2);
    u64 x = 1, m = 2ULL * (u64)n;
    for (int j = 0; j < n / 2; ++j) { e[j] = x; x = x * 5 % m; }
    return e;
}

void encode_poly(int n, const double *re, const double *im, size_t n_slots, double scale, i64 *out) {
    if (n_slots > (size_t)n / 2) throw Error(CKKS_E_INVALID_ARG, "more slots than N/2");
    std::vector<cd> v(n, cd(0, 0));
    auto e = slot_exponents(n);
    const u64 m2 = 2ULL * (u64)n;
    for (size_t j = 0; j < n_slots; ++j) {
        cd z(re ? re[j] * scale : 0.0, im ? im[j] * scale : 0.0);
        v[(e[j] - 1) / 2] = z;
        v[(m2 - e[j] - 1) / 2] = std::conj(z);
    }
    fft(v, -1);
    for (int i = 0; i < n; ++i) {
        double ang = -M_PI * (double)i / (double)n;
        double r = (v[i] * cd(std::cos(ang), std::sin(ang))).real() / (double)n;
        double rr = std::nearbyint(r);
        if (!(std::fabs(rr) < 4.6e18)) throw Error(CKKS_E_INVALID_ARG, "encoded coefficient too large");
        out[i] = (i64)rr;
    }
}

void decode_poly(int n, const double *coeffs, double *re, double *im) {
    std::vector<cd> t(n);
    for (int i = 0; i < n; ++i) {
        double ang = M_PI * (double)i / (double)n;
        t[i] = coeffs[i] * cd(std::cos(ang), std::sin(ang));
    }
    fft(t, +1);
    auto e = slot_exponents(n);
    for (int j = 0; j < n / 2; ++j) {
        cd z = t[(e[j] - 1) / 2];
        if (re) re[j] = z.real();
        if (im) im[j] = z.imag();
    }
}

// Block-start mask (1 at slots = 0 mod R): an R-periodic real vector, so it lies in the subring
// spanned by X^(c N / (2R)); its coefficient there is cos(pi c / (2R)) / R, c = 0..2R-1.  Times the
// scale and rounded half away from zero, in extended precision.
void mask_poly(int n, int R, double scale, i64 *out) {
    if (R < 1 || 2 * R > n || (R & (R - 1))) throw Error(CKKS_E_INVALID_ARG, "R must be a power of two <= N/2");
    const long double pi = 3.141592653589793238462643383279502884L;
    for (int i = 0; i < n; ++i) out[i] = 0;
    const int stride = n / (2 * R);
    for (int c = 0; c < 2 * R; ++c) {
        long double v = ((long double)scale * cosl(pi * (long double)c / (long double)(2 * R))) / (long double)R;
        out[c * stride] = (i64)llroundl(v);
    }
    out[R * stride] = 0;   // cos(pi / 2) is exactly zero
}

}  // namespace gck
