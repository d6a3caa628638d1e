// Spectral statistics of the emission spectra: the probe-summed power
// spectrum, its peak, its standard deviation and a Gaussian fit around the
// peak (the linewidth the Results section reads off the Maxwell-Bloch spectra
// by a Gaussian fit, Fig. 5b; the width of the experimental spectra is their
// standard deviation, Fig. 4).
//
//   S_k        = sum_p |F_{p,k}|^2                (probes summed in order)
//   peak       = argmax_k S_k                     (lowest k among equal maxima)
//   mean, std  = first moment and standard deviation of omega under S
//   fit window = the run of bins around the peak with S_k >= level * S_peak
//   fit        = weighted least-squares parabola ln(S_k / S_peak) = a + b x + c x^2
//                over the window, weights (S_k / S_peak)^2, x = (omega_k - omega_peak) / s,
//                s the mean bin spacing inside the window; a Gaussian has
//                c = -1/(2 sigma_x^2), centre x0 = -b/(2c), amplitude S_peak exp(a - b^2/(4c)).
#pragma once

#include "mbf_kernels.hpp"

namespace mbf {

constexpr int kStatThreads = 256;

// Sum over the workgroup in a fixed order, returned to every thread.
__device__ __forceinline__ double stat_sum(double x, double* sh) {
    const int t = (int)threadIdx.x;
    x = wave_sum(x);
    __syncthreads();                                  // earlier readers of sh are done
    if ((t & 63) == 0) sh[t >> 6] = x;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kStatThreads / 64; ++w) r += sh[w];
    return r;
}

// (value, bin) maximum with the lowest bin among equal values.
__device__ __forceinline__ void stat_max(double& v, int& k, double v2, int k2) {
    if (v2 > v || (v2 == v && k2 < k)) {
        v = v2;
        k = k2;
    }
}

// S_k = sum_p |F_{p,k}|^2, one thread per bin (a wave reads 64 consecutive
// complex values of one probe at a time); spec holds np x nf complex values,
// re and im interleaved, probe-major.  The probes are added in index order;
// the loads of eight probes go out before their sums.
__global__ void __launch_bounds__(64) k_spec_power(const double* __restrict__ spec, int np, int nf,
                                                   double* __restrict__ pw) {
    const int k = (int)(blockIdx.x * 64 + threadIdx.x);
    if (k >= nf) return;
    const double2* __restrict__ f = reinterpret_cast<const double2*>(spec);
    double s = 0.0;
    int p = 0;
    for (; p + 8 <= np; p += 8) {
        double2 v[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) v[q] = f[(int64_t)(p + q) * nf + k];
#pragma unroll
        for (int q = 0; q < 8; ++q) s += v[q].x * v[q].x + v[q].y * v[q].y;
    }
    for (; p < np; ++p) {
        const double2 v = f[(int64_t)p * nf + k];
        s += v.x * v.x + v.y * v.y;
    }
    pw[k] = s;
}

// One workgroup per spectrum: pw holds S (nf values, from k_spec_power),
// out receives the statistics.
__global__ void __launch_bounds__(kStatThreads) k_spec_stats(const double* __restrict__ pw, int nf,
                                                            const double* __restrict__ omega, double level,
                                                            mbf_spec_stats* out) {
    __shared__ double sh[kStatThreads / 64];
    __shared__ double shv[kStatThreads / 64];
    __shared__ int shk[kStatThreads / 64];
    __shared__ int win[2];
    const int t = (int)threadIdx.x;
    // ---- total, peak
    double tot = 0.0, best = -1.0;
    int bk = nf;
    for (int k = t; k < nf; k += kStatThreads) {
        const double s = pw[k];
        tot += s;
        stat_max(best, bk, s, k);
    }
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(best, o, 64);
        const int k2 = __shfl_xor(bk, o, 64);
        stat_max(best, bk, v2, k2);
    }
    if ((t & 63) == 0) {
        shv[t >> 6] = best;
        shk[t >> 6] = bk;
    }
    const double total = stat_sum(tot, sh);           // its barriers also publish shv and shk
    double peak = shv[0];
    int kp = shk[0];
    for (int w = 1; w < kStatThreads / 64; ++w) stat_max(peak, kp, shv[w], shk[w]);
    // ---- moments of omega under S
    double m1 = 0.0;
    for (int k = t; k < nf; k += kStatThreads) m1 += pw[k] * omega[k];
    const double mean = total > 0.0 ? stat_sum(m1, sh) / total : 0.0;
    double m2 = 0.0;
    for (int k = t; k < nf; k += kStatThreads) {
        const double d = omega[k] - mean;
        m2 += pw[k] * (d * d);
    }
    const double var = total > 0.0 ? stat_sum(m2, sh) / total : 0.0;
    // ---- fit window: the run around the peak above level * peak
    const double thr = level * peak;
    if (t == 0) {
        int lo = kp, hi = kp;
        if (total > 0.0) {
            while (lo > 0 && pw[lo - 1] >= thr) --lo;
            while (hi < nf - 1 && pw[hi + 1] >= thr) ++hi;
        }
        win[0] = lo;
        win[1] = hi;
    }
    __syncthreads();
    const int lo = win[0], hi = win[1];
    const bool can_fit = total > 0.0 && hi - lo >= 2 && omega[hi] != omega[lo];
    const double wp = can_fit ? omega[kp] : 0.0;
    const double s = can_fit ? (omega[hi] - omega[lo]) / (double)(hi - lo) : 1.0;
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0, a4 = 0.0, r0 = 0.0, r1 = 0.0, r2 = 0.0;
    if (can_fit) {
        for (int k = lo + t; k <= hi; k += kStatThreads) {
            const double x = (omega[k] - wp) / s;
            const double u = pw[k] / peak;
            const double w = u * u, y = log(u);
            const double x2 = x * x;
            a0 += w;
            a1 += w * x;
            a2 += w * x2;
            a3 += w * (x2 * x);
            a4 += w * (x2 * x2);
            r0 += w * y;
            r1 += w * (x * y);
            r2 += w * (x2 * y);
        }
        a0 = stat_sum(a0, sh); a1 = stat_sum(a1, sh); a2 = stat_sum(a2, sh);
        a3 = stat_sum(a3, sh); a4 = stat_sum(a4, sh);
        r0 = stat_sum(r0, sh); r1 = stat_sum(r1, sh); r2 = stat_sum(r2, sh);
    }
    if (t != 0) return;
    mbf_spec_stats o{};
    o.total = total;
    o.peak_bin = total > 0.0 ? kp : -1;
    o.peak_omega = total > 0.0 ? omega[kp] : 0.0;
    o.peak_value = total > 0.0 ? peak : 0.0;
    o.mean_omega = mean;
    o.std_omega = sqrt(var);
    o.fit_lo = total > 0.0 ? lo : -1;
    o.fit_hi = total > 0.0 ? hi : -1;
    o.fit_ok = 0;
    o.fit_center = o.fit_sigma = o.fit_amplitude = 0.0;
    if (can_fit) {
        // normal equations of the weighted parabola, by Cramer's rule
        const double d = a0 * (a2 * a4 - a3 * a3) - a1 * (a1 * a4 - a2 * a3) + a2 * (a1 * a3 - a2 * a2);
        const double da = r0 * (a2 * a4 - a3 * a3) - a1 * (r1 * a4 - a3 * r2) + a2 * (r1 * a3 - a2 * r2);
        const double db = a0 * (r1 * a4 - a3 * r2) - r0 * (a1 * a4 - a2 * a3) + a2 * (a1 * r2 - r1 * a2);
        const double dc = a0 * (a2 * r2 - r1 * a3) - a1 * (a1 * r2 - r1 * a2) + r0 * (a1 * a3 - a2 * a2);
        if (d != 0.0) {
            const double a = da / d, b = db / d, c = dc / d;
            if (c < 0.0) {
                o.fit_ok = 1;
                o.fit_center = wp + s * (-b / (2.0 * c));
                o.fit_sigma = fabs(s) * sqrt(-1.0 / (2.0 * c));
                o.fit_amplitude = peak * exp(a - b * b / (4.0 * c));
            }
        }
    }
    *out = o;
}

// Peaks of S (the long-lived modes of a passive spectrum, Fig. 1): bins with
// S_k > 0, S_k >= min_rel * max S, S_{k-1} < S_k >= S_{k+1} (an edge bin
// compares with its one neighbour; a flat top counts once, at its first bin),
// listed by decreasing S_k (equal values: lower k first), at most max_peaks.
// One workgroup; round r takes the largest candidate below the previous one
// in that order.
__global__ void __launch_bounds__(kStatThreads) k_spec_peaks(const double* __restrict__ pw, int nf, double min_rel,
                                                            int max_peaks, int32_t* __restrict__ bins,
                                                            int32_t* __restrict__ count) {
    __shared__ double sh[kStatThreads / 64];
    __shared__ double shv[kStatThreads / 64];
    __shared__ int shk[kStatThreads / 64];
    const int t = (int)threadIdx.x;
    double top = -1.0;
    int tk = nf;
    for (int k = t; k < nf; k += kStatThreads) stat_max(top, tk, pw[k], k);
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) {
        const double v2 = __shfl_xor(top, o, 64);
        const int k2 = __shfl_xor(tk, o, 64);
        stat_max(top, tk, v2, k2);
    }
    if ((t & 63) == 0) shv[t >> 6] = top;
    (void)stat_sum(0.0, sh);                          // barrier: shv published
    double smax = shv[0];
    for (int w = 1; w < kStatThreads / 64; ++w) smax = fmax(smax, shv[w]);
    const double thr = min_rel * smax;
    double pv = INFINITY;                             // previous pick (value, bin)
    int pk = -1;
    int found = 0;
    for (int r = 0; r < max_peaks; ++r) {
        double best = -1.0;
        int bk = nf;
        for (int k = t; k < nf; k += kStatThreads) {
            const double v = pw[k];
            const bool is_peak = v > 0.0 && v >= thr && (k == 0 || pw[k - 1] < v) && (k == nf - 1 || v >= pw[k + 1]);
            const bool below = v < pv || (v == pv && k > pk);
            if (is_peak && below) stat_max(best, bk, v, k);
        }
#pragma unroll
        for (int o = 32; o > 0; o >>= 1) {
            const double v2 = __shfl_xor(best, o, 64);
            const int k2 = __shfl_xor(bk, o, 64);
            stat_max(best, bk, v2, k2);
        }
        __syncthreads();                              // readers of the previous round are done
        if ((t & 63) == 0) {
            shv[t >> 6] = best;
            shk[t >> 6] = bk;
        }
        __syncthreads();
        best = shv[0];
        bk = shk[0];
        for (int w = 1; w < kStatThreads / 64; ++w) stat_max(best, bk, shv[w], shk[w]);
        if (best < 0.0) break;                        // uniform: no candidate left
        if (t == 0) bins[r] = bk;
        pv = best;
        pk = bk;
        found = r + 1;
    }
    if (t == 0) *count = found;
}

// ---------------------------------------------------------------- threshold
// Growth rate of one run of a pump sweep (one workgroup per run): the
// least-squares slope of ln W^n against n over n0 <= n < n1, formed about the
// window's centre nc = (n0 + n1 - 1)/2, where sum (n - nc) = 0:
//   rate = sum (n - nc) ln W^n / sum (n - nc)^2,
// the denominator in closed form, m (m^2 - 1) / 12 for m = n1 - n0 steps.  A
// non-positive W gives NaN.
__global__ void __launch_bounds__(kStatThreads) k_growth_rate(const double* const* __restrict__ hist, int64_t n0,
                                                            int64_t n1, double* __restrict__ rates) {
    __shared__ double sh[kStatThreads / 64];
    const double* __restrict__ w = hist[blockIdx.x];
    const double nc = 0.5 * (double)(n0 + n1 - 1);
    double s = 0.0;
    for (int64_t n = n0 + (int64_t)threadIdx.x; n < n1; n += kStatThreads) {
        const double x = w[n];
        s += ((double)n - nc) * (x > 0.0 ? log(x) : __builtin_nan(""));
    }
    s = stat_sum(s, sh);
    if (threadIdx.x == 0) {
        const double m = (double)(n1 - n0);
        rates[blockIdx.x] = s / (m * (m * m - 1.0) / 12.0);
    }
}

// The least-squares line rate = a + b N_a through a sweep of R runs and its
// root N_th = -a/b (one thread; R is small): fit = (a, b, N_th).
__global__ void k_threshold_line(const double* __restrict__ Na, const double* __restrict__ rates, int R,
                                 double* __restrict__ fit) {
    if (threadIdx.x != 0 || blockIdx.x != 0) return;
    double mx = 0.0, my = 0.0;
    for (int r = 0; r < R; ++r) {
        mx += Na[r];
        my += rates[r];
    }
    mx /= R;
    my /= R;
    double sxy = 0.0, sxx = 0.0;
    for (int r = 0; r < R; ++r) {
        sxy += (Na[r] - mx) * (rates[r] - my);
        sxx += (Na[r] - mx) * (Na[r] - mx);
    }
    const double b = sxy / sxx;
    const double a = my - b * mx;
    fit[0] = a;
    fit[1] = b;
    fit[2] = -a / b;
}

// ------------------------------------------------ knee of a pump sweep
// Two straight lines fitted to y against x (x increasing), joined at a knee:
// for every split s, with points [0, s) and [s, n) at least two each, the
// least-squares line of each part (centred sums in index order) and the sum
// of the two parts' squared residuals; the split with the smallest sum (the
// first on ties) and the crossing of its two lines, kept between x[s-1] and
// x[s] (their midpoint when the lines do not cross there at a finite point).
// One workgroup; out: knee, s, aL, bL, aR, bR, residual sum.
constexpr int kKneeMax = 1024;

struct KneeLine {
    double a, b, sse;
};

__device__ inline KneeLine knee_line(const double* __restrict__ x, const double* __restrict__ y, int i0, int i1) {
    const double m = (double)(i1 - i0);
    double mx = 0.0, my = 0.0;
    for (int i = i0; i < i1; ++i) {
        mx += x[i];
        my += y[i];
    }
    mx /= m;
    my /= m;
    double sxy = 0.0, sxx = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double dx = x[i] - mx;
        sxy += dx * (y[i] - my);
        sxx += dx * dx;
    }
    KneeLine l;
    l.b = sxy / sxx;
    l.a = my - l.b * mx;
    l.sse = 0.0;
    for (int i = i0; i < i1; ++i) {
        const double r = y[i] - (l.a + l.b * x[i]);
        l.sse += r * r;
    }
    return l;
}

__global__ void __launch_bounds__(256) k_knee_fit(const double* __restrict__ x, const double* __restrict__ y, int n,
                                                  double* __restrict__ out) {
    __shared__ double s_sse[kKneeMax];
    for (int s = 2 + (int)threadIdx.x; s <= n - 2; s += (int)blockDim.x) {
        const KneeLine L = knee_line(x, y, 0, s), R = knee_line(x, y, s, n);
        s_sse[s] = L.sse + R.sse;
    }
    __syncthreads();
    if (threadIdx.x != 0) return;
    int best = 2;
    for (int s = 3; s <= n - 2; ++s)
        if (s_sse[s] < s_sse[best]) best = s;
    const KneeLine L = knee_line(x, y, 0, best), R = knee_line(x, y, best, n);
    const double lo = x[best - 1], hi = x[best];
    double k = (R.a - L.a) / (L.b - R.b);
    if (!isfinite(k)) k = 0.5 * (lo + hi);
    k = fmin(fmax(k, lo), hi);
    out[0] = k;
    out[1] = (double)best;
    out[2] = L.a;
    out[3] = L.b;
    out[4] = R.a;
    out[5] = R.b;
    out[6] = s_sse[best];
}

}  // namespace mbf
