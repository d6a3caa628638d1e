// Bound states of the dimensionless Gross-Pitaevskii equation of the random
// laser (the oscillation condition gain = loss with gain saturation, finite
// gain bandwidth and a quadratic trap from the high-Q modes, Gross-Pitaevskii
// section, Eq. g5):
//
//     -phi'' + tau^2 phi + phi^3 = E phi,     phi(tau) > 0, phi -> 0 at |tau| -> inf,
//
// for a batch of nonlinear eigenvalues E > 1, and the normalised spectrum of
// each solution (its Fourier transform, Eq. s1 and Fig. 5: waist and peak).
//
// Discretisation: M interior points tau_i = -L + (i+1) h, h = 2L/(M+1),
// phi = 0 at tau = +-L, second differences.  Each E is solved by one
// workgroup: a semi-implicit gradient flow
//     (A + diag(phi_k^2) - E + 1/ds) phi_{k+1} = phi_k / ds,   ds = 1/E
// (A = -d2 + tau^2; an M-matrix, so phi stays positive), then Newton steps
//     (A + diag(3 phi^2) - E) delta = -(A phi + phi^3 - E phi)
// until the update is below 1e-13 of max phi.  Every tridiagonal system is
// solved by parallel cyclic reduction in LDS.  The spectrum is
//     phit(nu) = (h / 2 pi) sum_i phi_i cos(nu tau_i),  S(nu) = phit(nu)^2
// on nu_k = k dnu; its peak is S(0) and its waist w = sigma_nu / (2 pi),
// sigma_nu^2 the second moment of the symmetric spectrum (S_0 + 2 sum_{k>=1}
// weights), so that a Gaussian S ~ exp(-nu^2 / (8 pi^2 w^2)) has waist w.
#pragma once

#include "mbf_kernels.hpp"

namespace mbf {

constexpr int kGpThreads = 256;
constexpr int kGpMaxM = 1023;          // interior points (padded to 1024 for the reduction)
constexpr int kGpP = 1024;

// Sum over the workgroup in a fixed order, returned to every thread.
__device__ __forceinline__ double gp_sum(double x, double* sh) {
    const int t = (int)threadIdx.x;
    x = wave_sum(x);
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = x;
    __syncthreads();
    double r = 0.0;
#pragma unroll
    for (int w = 0; w < kGpThreads / 64; ++w) r += sh[w];
    return r;
}

__device__ __forceinline__ double gp_max(double x, double* sh) {
    const int t = (int)threadIdx.x;
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x = fmax(x, __shfl_xor(x, o, 64));
    __syncthreads();
    if ((t & 63) == 0) sh[t >> 6] = x;
    __syncthreads();
    double r = sh[0];
#pragma unroll
    for (int w = 1; w < kGpThreads / 64; ++w) r = fmax(r, sh[w]);
    return r;
}

// Parallel cyclic reduction of the tridiagonal system (a_i x_{i-1} + b_i x_i
// + c_i x_{i+1} = d_i) held in LDS over kGpP rows (rows past the system are
// identity rows); on return d_i / b_i is x_i.  Every row is reduced against
// its neighbours at distance s = 1, 2, 4, ...
__device__ __forceinline__ void gp_pcr(double* a, double* b, double* c, double* d) {
    constexpr int R = kGpP / kGpThreads;
    const int t = (int)threadIdx.x;
    for (int s = 1; s < kGpP; s <<= 1) {
        double na[R], nb[R], nc[R], nd[R];
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kGpThreads;
            const int lo = i - s, hi = i + s;
            const double al = lo >= 0 ? -a[i] / b[lo] : 0.0;
            const double ga = hi < kGpP ? -c[i] / b[hi] : 0.0;
            na[r] = lo >= 0 ? al * a[lo] : 0.0;
            nc[r] = hi < kGpP ? ga * c[hi] : 0.0;
            nb[r] = b[i] + (lo >= 0 ? al * c[lo] : 0.0) + (hi < kGpP ? ga * a[hi] : 0.0);
            nd[r] = d[i] + (lo >= 0 ? al * d[lo] : 0.0) + (hi < kGpP ? ga * d[hi] : 0.0);
        }
        __syncthreads();
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kGpThreads;
            a[i] = na[r];
            b[i] = nb[r];
            c[i] = nc[r];
            d[i] = nd[r];
        }
        __syncthreads();
    }
}

struct GpArgs {
    const double* E;       // n_E eigenvalues
    int M;                 // interior points (3 .. kGpMaxM)
    double L;              // half-width of the tau window
    int n_nu;              // spectrum points nu_k = k dnu
    double dnu;
    int flow_iters;        // gradient-flow steps before Newton
    int newton_iters;      // Newton steps at most
    double* phi;           // n_E x M
    double* spec;          // n_E x n_nu
    double* stats;         // n_E x kGpStats
};

// stats per E: N = h sum phi^2, w, p = S(0), phi(0) (largest sample), max
// residual |A phi + phi^3 - E phi|, Newton steps taken, 1 when converged
constexpr int kGpStats = 7;

__global__ void __launch_bounds__(kGpThreads) k_gp_solve(GpArgs g) {
    __shared__ double a[kGpP], b[kGpP], c[kGpP], d[kGpP];
    __shared__ double ph[kGpP];
    __shared__ double sh[kGpThreads / 64];
    constexpr int R = kGpP / kGpThreads;
    const int t = (int)threadIdx.x;
    const int e = (int)blockIdx.x;
    const double E = g.E[e];
    const int M = g.M;
    const double h = 2.0 * g.L / (double)(M + 1);
    const double ih2 = 1.0 / (h * h);
    const double ds = 1.0 / E;
    // initial profile: the near-threshold Gaussian for E < 3, Thomas-Fermi above
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * kGpThreads;
        double v = 0.0;
        if (i < M) {
            const double tau = -g.L + (double)(i + 1) * h;
            v = E < 3.0 ? sqrt(sqrt(2.0) * (E - 1.0)) * exp(-0.5 * tau * tau) : sqrt(fmax(E - tau * tau, 0.0) + 1e-3);
        }
        ph[i] = v;
    }
    __syncthreads();
    // gradient flow
    for (int it = 0; it < g.flow_iters; ++it) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kGpThreads;
            if (i < M) {
                const double tau = -g.L + (double)(i + 1) * h;
                a[i] = i > 0 ? -ih2 : 0.0;
                c[i] = i < M - 1 ? -ih2 : 0.0;
                b[i] = 2.0 * ih2 + tau * tau + ph[i] * ph[i] - E + 1.0 / ds;
                d[i] = ph[i] / ds;
            } else {
                a[i] = 0.0; b[i] = 1.0; c[i] = 0.0; d[i] = 0.0;
            }
        }
        __syncthreads();
        gp_pcr(a, b, c, d);
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kGpThreads;
            ph[i] = i < M ? d[i] / b[i] : 0.0;
        }
        __syncthreads();
    }
    // Newton
    int steps = 0;
    int converged = 0;
    for (int it = 0; it < g.newton_iters; ++it) {
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kGpThreads;
            if (i < M) {
                const double tau = -g.L + (double)(i + 1) * h;
                const double p = ph[i];
                const double pl = i > 0 ? ph[i - 1] : 0.0, pr = i < M - 1 ? ph[i + 1] : 0.0;
                const double F = (2.0 * p - pl - pr) * ih2 + tau * tau * p + p * p * p - E * p;
                a[i] = i > 0 ? -ih2 : 0.0;
                c[i] = i < M - 1 ? -ih2 : 0.0;
                b[i] = 2.0 * ih2 + tau * tau + 3.0 * p * p - E;
                d[i] = -F;
            } else {
                a[i] = 0.0; b[i] = 1.0; c[i] = 0.0; d[i] = 0.0;
            }
        }
        __syncthreads();
        gp_pcr(a, b, c, d);
        double dmax = 0.0, pmax = 0.0;
#pragma unroll
        for (int r = 0; r < R; ++r) {
            const int i = t + r * kGpThreads;
            if (i < M) {
                const double dl = d[i] / b[i];
                ph[i] += dl;
                dmax = fmax(dmax, fabs(dl));
                pmax = fmax(pmax, fabs(ph[i]));
            }
        }
        dmax = gp_max(dmax, sh);
        pmax = gp_max(pmax, sh);
        steps = it + 1;
        if (dmax <= 1e-13 * pmax) {
            converged = 1;
            break;
        }
    }
    __syncthreads();
    // residual, norm, output profile
    double res = 0.0, nrm = 0.0, pk = 0.0;
#pragma unroll
    for (int r = 0; r < R; ++r) {
        const int i = t + r * kGpThreads;
        if (i < M) {
            const double tau = -g.L + (double)(i + 1) * h;
            const double p = ph[i];
            const double pl = i > 0 ? ph[i - 1] : 0.0, pr = i < M - 1 ? ph[i + 1] : 0.0;
            res = fmax(res, fabs((2.0 * p - pl - pr) * ih2 + tau * tau * p + p * p * p - E * p));
            nrm += p * p;
            pk = fmax(pk, p);
            g.phi[(int64_t)e * M + i] = p;
        }
    }
    res = gp_max(res, sh);
    pk = gp_max(pk, sh);
    nrm = h * gp_sum(nrm, sh);
    // spectrum: one frequency per thread at a time, the sum over tau in order
    double s0 = 0.0, s2 = 0.0, peak = 0.0;
    for (int k = t; k < g.n_nu; k += kGpThreads) {
        const double nu = (double)k * g.dnu;
        double f = 0.0;
        for (int i = 0; i < M; ++i) f += ph[i] * cos(nu * (-g.L + (double)(i + 1) * h));
        f *= h / (2.0 * 3.14159265358979323846);
        const double S = f * f;
        g.spec[(int64_t)e * g.n_nu + k] = S;
        const double wgt = k == 0 ? 1.0 : 2.0;    // the spectrum is even in nu
        s0 += wgt * S;
        s2 += wgt * S * nu * nu;
        if (k == 0) peak = S;
    }
    s0 = gp_sum(s0, sh);
    s2 = gp_sum(s2, sh);
    peak = gp_sum(peak, sh);
    if (t == 0) {
        double* st = g.stats + (int64_t)e * kGpStats;
        st[0] = nrm;
        st[1] = s0 > 0.0 ? sqrt(s2 / s0) / (2.0 * 3.14159265358979323846) : 0.0;
        st[2] = peak;
        st[3] = pk;
        st[4] = res;
        st[5] = (double)steps;
        st[6] = (double)converged;
    }
}

}  // namespace mbf
