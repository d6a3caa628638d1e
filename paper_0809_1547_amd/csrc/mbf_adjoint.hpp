// Device code of the adjoint (reverse) step of the Maxwell-Bloch FDTD step.
//
// Objective: L = sum over steps n = 1..N of sum over the interior E-sites of
// the loss box of (E^n)^2.  The forward step X^{n+1} = F(X^n; eps, N_a) is
// linearised at the stored trajectory and its transpose is applied backwards.
// Writing etot for the total adjoint of E^{n+1} (its later uses plus the
// work term W of step n), the reverse step is
//   H-sites:  htot = da * htot_prev + S curl+(u),  u = cb ie etot on interior
//             E-sites, zero elsewhere (the transpose of curl- is curl+)
//   E-sites:  lambda_E^n = ca etot - S curl-(db htot) + Bloch terms + 2 E^n
//             in the box (the transpose of curl+ is curl-),
// and the E part stores u rather than etot, so that the H part reads plain
// values like the forward a1.
// with the transposed Lorentz-oscillator and rate-equation Jacobians at the
// gain sites, and the parameter terms
//   dL/d eps(cell) += etot . (E^{n+1} - ca E^n - src) . (-1/eps)  (E' depends
//   on eps through ie = 1/eps), and dL/dN_a from the pump term of N3 and the
//   noise amplitude c_F = ck N_a E_sp.
// The populations carry N1..N3 (N0 = N_a - N1 - N2 - N3), as in the forward
// kernels.  Wall sites are constant and never feed a parameter, so they are
// skipped; H-sites outside [0,n)^3 are never used.
#pragma once

#include "mbf_kernels.hpp"

namespace mbf {

template <typename T>
struct AdjView {
    using value_type = T;
    // forward trajectory: slot q = m - ctl->tap_base of `slot` values holds
    // E^m (3 x tap_e dense), P^m - P^{m-1} (3 x tap_c compact) and N1^m - N2^m
    // (3 x tap_c compact); a reverse step is told its slot q and takes back
    // step n = ctl->tap_base + q, so one captured sequence of reverse steps
    // serves every segment
    const T* traj;
    int64_t slot, tap_e, tap_c;
    Ctl* ctl;
    // adjoint state, updated in place
    T* u[3];             // in: cb ie etot of E^{n+1}; out: of E^n (for step n-1); zero off the interior
    T* hb[3];            // htot of the previous reverse step on entry, of this one on exit
    T* lp[3];            // adjoint of P^{n+1} in, of P^n out (compact)
    T* lq[3];            // adjoint of the P^n copy (P_prev slot of step n+1) in, of P^{n-1} out
    T* ln[3][3];         // adjoint of N1..N3 at n+1 in, at n out
    double* g_eps;       // dL/d eps per cell, x fastest (nx*ny*nz)
    double* g_na;        // per work item partial sums of dL/d(N_a/N_ref)
    // material and geometry
    const uint8_t* mat;
    const uint32_t* seg_base;
    int nbx;
    const T* lut_inv_eps;
    int nx, ny, nz;
    int64_t sx, sxy;
    int has_layer;            // lossy-layer coefficient table, as in SimView
    const uint8_t* lev[3][2];
    const T* lc;
    uint32_t lc_sy, lc_sz;
    // coefficients of the forward step
    T S, a, b, ck, beta, dt32, dt21, dt10, dtWp;
    T ck_esp;            // d c_F / d(N_a/N_ref) = ck E_sp (0 without noise)
    int noise;
    uint32_t seed_lo, seed_hi, realization;
    // soft source of the forward run (its value at step n is formed again)
    int src_on, src_kind, src_comp, src_i, src_j, src_k;
    double src_amp, src_ws, src_tp, src_t0, dt;
    int box[6];
};

// Trajectory slots q and q+1 (steps n and n+1, n = ctl->tap_base + q).
template <typename T>
struct AdjSlot {
    const T* s0;
    const T* s1;
    int64_t n;
};

template <typename T>
__device__ __forceinline__ AdjSlot<T> adj_slot(const AdjView<T>& v, int q) {
    AdjSlot<T> a;
    a.n = gld(&v.ctl->tap_base) + q;
    a.s0 = v.traj + (int64_t)q * v.slot;
    a.s1 = a.s0 + v.slot;
    return a;
}

// Interior E-site test (updated by Ampere's law).
template <typename T>
__device__ __forceinline__ bool e_in(const AdjView<T>& v, int c, int i, int j, int k) {
    const bool ox = c == 0 ? (i >= 0 && i < v.nx) : (i >= 1 && i < v.nx);
    const bool oy = c == 1 ? (j >= 0 && j < v.ny) : (j >= 1 && j < v.ny);
    const bool oz = c == 2 ? (k >= 0 && k < v.nz) : (k >= 1 && k < v.nz);
    return ox && oy && oz;
}


// H part: htot = da htot_prev + S curl+(u) on the H-sites of [0,n)^3.
// The view of a run lives in device memory and is read through a no-alias
// pointer (constant over the run), so its fields stay out of the kernel
// arguments and scalar registers.
template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY) k_adj_h(const AdjView<T>* __restrict__ vp, Geom gm) {
    const AdjView<T>& v = *vp;
    int bx, by, bz;
    decode_item(gm, xcd_work_item((int)blockIdx.x, gm.nblk, gm.xcd_remap), bx, by, bz);
    const int i = bx * 64 + threadIdx.x;
    const int j = by * TY + threadIdx.y;
    if (i >= v.nx || j >= v.ny) return;
    const int kz0 = bz * gm.zseg, kz1 = min(kz0 + gm.zseg, v.nz);
    const uint32_t sx = (uint32_t)v.sx, sxy = (uint32_t)v.sxy;
    const T* __restrict__ ux = v.u[0];
    const T* __restrict__ uy = v.u[1];
    const T* __restrict__ uz = v.u[2];
    for (int k = kz0; k < kz1; ++k) {
        const uint32_t x = (uint32_t)i + sx * (uint32_t)j + sxy * (uint32_t)k;
        const T cx = (ldo(uz, x + sx) - ldo(uz, x)) - (ldo(uy, x + sxy) - ldo(uy, x));
        const T cy = (ldo(ux, x + sxy) - ldo(ux, x)) - (ldo(uz, x + 1u) - ldo(uz, x));
        const T cz = (ldo(uy, x + 1u) - ldo(uy, x)) - (ldo(ux, x + sx) - ldo(ux, x));
        const T cc[3] = {cx, cy, cz};
#pragma unroll
        for (int c = 0; c < 3; ++c) {
            const T da = lay_coef_h(v, c, i, j, k).ca;
            sto(v.hb[c], x, da * ldo(v.hb[c], x) + v.S * cc[c]);
        }
    }
}

// Everything the E part reads for one plane of a row: htot at the cell's own
// H-sites and at the y-1 and x-1 neighbours its curl- needs (z-1 is carried
// from the previous plane), u, E^n and E^{n+1} of the three E-sites, the
// Bloch trajectory and adjoint state of the gain sites, and the cell's eps
// gradient so far.  Loaded ahead of the plane's stores (the arrays may share
// no memory, but the compiler cannot know that through the view).
template <typename T>
struct AdjPlane {
    T hx, hy, hz, hz_y, hx_y, hz_x, hy_x;
    T u[3], E[3], En[3];
    T dPf[3], dN[3], n1[3], n2[3], n3[3], lp[3], lq[3], dPp[3];
    double ge;
};

// Lanes past the grid read column nx and cell 0 (valid sites; their values
// are not used); the y-1 and x-1 neighbours only exist for j >= 1 and i >= 1
// (the offsets would wrap below zero otherwise).
template <typename T>
__device__ __forceinline__ void adj_load_plane(AdjPlane<T>& p, const AdjView<T>& v, const AdjSlot<T>& a, uint32_t x,
                                               uint32_t cell, uint32_t gi, bool g, int i, int j, int k) {
    const uint32_t sx = (uint32_t)v.sx;
    p.hx = ldo(v.hb[0], x); p.hy = ldo(v.hb[1], x); p.hz = ldo(v.hb[2], x);
    p.hz_y = j >= 1 ? ldo(v.hb[2], x - sx) : (T)0;
    p.hx_y = j >= 1 ? ldo(v.hb[0], x - sx) : (T)0;
    p.hz_x = i >= 1 ? ldo(v.hb[2], x - 1u) : (T)0;
    p.hy_x = i >= 1 ? ldo(v.hb[1], x - 1u) : (T)0;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        p.u[c] = ldo(v.u[c], x);
        p.E[c] = ldo(a.s0 + c * v.tap_e, x);
        p.En[c] = ldo(a.s1 + c * v.tap_e, x);
        const bool gs = g && e_in(v, c, i, j, k);
        p.dPf[c] = gs ? ldo(a.s1 + 3 * v.tap_e + c * v.tap_c, gi) : (T)0;
        p.dN[c] = gs ? ldo(a.s0 + 3 * v.tap_e + (3 + c) * v.tap_c, gi) : (T)0;
        p.n1[c] = gs ? ldo(v.ln[0][c], gi) : (T)0;
        p.n2[c] = gs ? ldo(v.ln[1][c], gi) : (T)0;
        p.n3[c] = gs ? ldo(v.ln[2][c], gi) : (T)0;
        p.lp[c] = gs ? ldo(v.lp[c], gi) : (T)0;
        p.lq[c] = gs ? ldo(v.lq[c], gi) : (T)0;
        p.dPp[c] = gs ? ldo(a.s0 + 3 * v.tap_e + c * v.tap_c, gi) : (T)0;
    }
    p.ge = gld(v.g_eps + cell);
}

// db htot at H-site c of (i, j, k) from its loaded htot.
template <typename T>
__device__ __forceinline__ T adj_db(const AdjView<T>& v, int c, int i, int j, int k, T hb) {
    return lay_coef_h(v, c, i, j, k).cb * hb;
}

// E part with the Bloch terms, the parameter terms and the loss term.  Each
// wave owns one row and marches along z (htot of Hx, Hy at k-1 stays in
// registers); a plane's loads all go out before its arithmetic and stores.
template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY) k_adj_e(const AdjView<T>* __restrict__ vp, Geom gm, int q) {
    const AdjView<T>& v = *vp;
    __shared__ double sh[TY];
    const int w = xcd_work_item((int)blockIdx.x, gm.nblk, gm.xcd_remap);
    int bx, by, bz;
    decode_item(gm, w, bx, by, bz);
    const int i = bx * 64 + threadIdx.x;
    const int j = by * TY + threadIdx.y;
    const int kz0 = bz * gm.zseg, kz1 = min(kz0 + gm.zseg, v.nz);
    const AdjSlot<T> a = adj_slot(v, q);
    const T src = v.src_on ? (T)source_at(v, a.n) : (T)0;   // the forward's value at step n
    double gna = 0.0;
    if (j < v.ny) {
        const bool act = i < v.nx;
        const uint32_t sxy = (uint32_t)v.sxy;
        const uint32_t pcell = (uint32_t)v.nx * (uint32_t)v.ny;
        uint32_t x = (uint32_t)(act ? i : v.nx) + (uint32_t)v.sx * (uint32_t)j + sxy * (uint32_t)kz0;
        uint32_t cell = (uint32_t)(act ? i : 0) + (uint32_t)v.nx * ((uint32_t)j + (uint32_t)v.ny * (uint32_t)kz0);
        uint8_t m = ldo(v.mat, x);
        uint32_t gi = gain_index(v, bx, j, kz0, act && m >= kGainId, true);
        uint8_t m_n = (kz0 + 1 < kz1) ? ldo(v.mat, x + sxy) : (uint8_t)0;
        // db htot of Hx, Hy at plane k-1, carried along z
        T vhx_z = (T)0, vhy_z = (T)0;
        if (act && kz0 >= 1) {
            vhx_z = adj_db(v, 0, i, j, kz0 - 1, ldo(v.hb[0], x - sxy));
            vhy_z = adj_db(v, 1, i, j, kz0 - 1, ldo(v.hb[1], x - sxy));
        }
        for (int k = kz0; k < kz1; ++k, x += sxy, cell += pcell) {
            AdjPlane<T> P;
            adj_load_plane(P, v, a, x, cell, gi, act && m >= kGainId, i, j, k);
            uint32_t gi_n = 0;
            uint8_t m_nn = 0;
            if (k + 1 < kz1) {
                gi_n = gain_index(v, bx, j, k + 1, act && m_n >= kGainId, true);
                if (k + 2 < kz1) m_nn = ldo(v.mat, x + 2u * sxy);
            }
            const bool g = act && m >= kGainId;
            const T vhx = adj_db(v, 0, i, j, k, P.hx);
            const T vhy = adj_db(v, 1, i, j, k, P.hy);
            if (act) {
                const T vhz = adj_db(v, 2, i, j, k, P.hz);
                const T ie = gld(v.lut_inv_eps + m);
                double geps = 0.0;
                T xi[3] = {(T)0, (T)0, (T)0};
                if (g && v.noise) noise3(v, cell, (uint32_t)a.n, xi);
#pragma unroll
                for (int c = 0; c < 3; ++c) {
                    if (!e_in(v, c, i, j, k)) continue;
                    T curl;
                    if (c == 0)
                        curl = (vhz - adj_db(v, 2, i, j - 1, k, P.hz_y)) - (vhy - vhy_z);
                    else if (c == 1)
                        curl = (vhx - vhx_z) - (vhz - adj_db(v, 2, i - 1, j, k, P.hz_x));
                    else
                        curl = (vhy - adj_db(v, 1, i - 1, j, k, P.hy_x)) - (vhx - adj_db(v, 0, i, j - 1, k, P.hx_y));
                    const LayC<T> lay = lay_coef_e(v, c, i, j, k);
                    const T ca = lay.ca, cb = lay.cb;
                    const T et = P.u[c] / (cb * ie);
                    const T E = P.E[c], En = P.En[c];
                    T lam = ca * et - v.S * curl;
                    T Wh_prev = (T)0, dP_prev = (T)0;
                    if (g) {
                        const T dPf = P.dPf[c];
                        const T dN = P.dN[c];
                        const T n1 = P.n1[c], n2 = P.n2[c], n3 = P.n3[c];
                        const T Wh = n2 - n1;
                        const T dPh = Wh * v.beta * (T)0.5 * (En + E) - cb * ie * et;
                        const T pn = P.lp[c] + dPh;
                        lam += v.ck * dN * pn + Wh * v.beta * (T)0.5 * dPf;
                        sto(v.lp[c], gi, P.lq[c] + v.a * pn - dPh);
                        sto(v.lq[c], gi, v.b * pn);
                        const T m1 = n1 * ((T)1 - v.dt10) - n3 * v.dtWp + v.ck * E * pn;
                        const T m2 = n2 * ((T)1 - v.dt21) + n1 * v.dt21 - n3 * v.dtWp - v.ck * E * pn;
                        const T m3 = n3 * ((T)1 - v.dt32 - v.dtWp) + n2 * v.dt32;
                        sto(v.ln[0][c], gi, m1);
                        sto(v.ln[1][c], gi, m2);
                        sto(v.ln[2][c], gi, m3);
                        gna += (double)(n3 * v.dtWp) + (double)(v.ck_esp * xi[c] * pn);
                        Wh_prev = m2 - m1;
                        dP_prev = P.dPp[c];
                    }
                    // E^{n+1} = ca E^n + cb ie (S curl- H' - dP) + src: its eps derivative
                    const T s = (v.src_on && c == v.src_comp && i == v.src_i && j == v.src_j && k == v.src_k) ? src : (T)0;
                    geps += (double)et * (double)((En - ca * E) - s) * (double)(-ie);
                    // loss term of E^n and the work term of step n-1
                    if (a.n >= 1) {
                        if (i >= v.box[0] && i < v.box[3] && j >= v.box[1] && j < v.box[4] && k >= v.box[2] && k < v.box[5])
                            lam += (T)2 * E;
                        lam += Wh_prev * v.beta * (T)0.5 * dP_prev;
                    }
                    sto(v.u[c], x, cb * ie * lam);
                }
                sto(v.g_eps, cell, P.ge + geps);
            }
            vhx_z = vhx;
            vhy_z = vhy;
            m = m_n;
            m_n = m_nn;
            gi = gi_n;
        }
    }
    const double s = block_sum(gna, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) sto(v.g_na, (uint32_t)w, gld(v.g_na + w) + s);
}

// Start of the reverse sweep: etot = 2 E^N on the interior sites of the box
// (u = cb ie etot; zero elsewhere); the other adjoint arrays start at zero.
template <typename T>
__global__ void __launch_bounds__(64) k_adj_seed(AdjView<T> v, int q) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    if (i > v.nx) return;
    const uint32_t x = (uint32_t)i + (uint32_t)v.sx * (uint32_t)j + (uint32_t)v.sxy * (uint32_t)k;
    const bool inb = i >= v.box[0] && i < v.box[3] && j >= v.box[1] && j < v.box[4] && k >= v.box[2] && k < v.box[5];
    const AdjSlot<T> a = adj_slot(v, q);              // q = N - 1 - tap_base: slot q+1 holds E^N
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        T u = (T)0;
        if (inb && e_in(v, c, i, j, k)) {
            const T ie = gld(v.lut_inv_eps + ldo(v.mat, x));
            const T cb = lay_coef_e(v, c, i, j, k).cb;
            u = cb * ie * ((T)2 * ldo(a.s1 + c * v.tap_e, x));
        }
        sto(v.u[c], x, u);
    }
}

// dL/d(N_a/N_ref) through the initial populations N_i^0 = r_i N_a/N_ref of
// the prepumped start: per-work-item partials of sum r_i lambda_Ni^0.
template <typename T>
__global__ void __launch_bounds__(64) k_adj_init_pop(AdjView<T> v, double r1, double r2, double r3, double* part) {
    __shared__ double sh[1];
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    const bool act = i < v.nx;
    const uint32_t x = (uint32_t)(act ? i : 0) + (uint32_t)v.sx * (uint32_t)j + (uint32_t)v.sxy * (uint32_t)k;
    const bool g = act && ldo(v.mat, x) >= kGainId;
    const uint32_t gi = gain_index(v, (int)blockIdx.x, j, k, g, true);
    double acc = 0.0;
    if (g) {
#pragma unroll
        for (int c = 0; c < 3; ++c)
            if (e_in(v, c, i, j, k))
                acc += r1 * (double)ldo(v.ln[0][c], gi) + r2 * (double)ldo(v.ln[1][c], gi) + r3 * (double)ldo(v.ln[2][c], gi);
    }
    const double s = block_sum(acc, sh);
    if (threadIdx.x == 0) part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
}

}  // namespace mbf
