// Device code of the Maxwell-Bloch FDTD step for gfx950 (wave64).
//
// Layout: every field component is a structure-of-arrays array over the
// extended Yee index range (nx+1)*(ny+1)*(nz+1), x fastest.  E and H are
// double-buffered (the step reads buffer `par` and writes buffer `par^1`,
// par = step & 1), so a kernel never reads a value another workgroup of the
// same launch may already have overwritten.  P keeps P^n and P^{n-1}; P^{n+1}
// is written over P^{n-1}.  N1..N3 are updated in place (each site only reads
// itself).  Material is one byte per site: an index into a small table of
// (1/eps_r, eps_r, Mur coefficient, gain flag).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbf {

constexpr int kBlockX = 64;   // one wave along x
constexpr int kBlockY = 4;    // four waves per workgroup
constexpr int kThreads = kBlockX * kBlockY;
constexpr int kMaxMat = 256;
constexpr int kMaxMurTasks = 12;

struct Ctl {                  // per-simulation control block (device memory)
    int64_t step;             // steps taken since the pump was set
    double W_now;             // energy of the last step
    double W_int;             // sum of the energy over all steps
    double loss;              // loss-box integral
    int32_t nonfinite;        // set once a step produced a non-finite energy
    int32_t pad;
};

template <typename T>
struct SimView {
    T* E[2][3];
    T* H[2][3];
    T* P[2][3];
    T* N[3][3];               // N1, N2, N3 x component
    const uint8_t* mat;       // per site of the extended range
    const T* lut_inv_eps;     // per material id
    const T* lut_eps;
    const T* lut_mur;
    const uint8_t* lut_gain;
    int nx, ny, nz;
    int64_t sx, sxy;          // strides of the extended range
    T S, a, b, ck, cF, beta, dt32, dt21, dt10, dtWp, Na;
    int noise;
    int frozen_pop;
    uint32_t seed_lo, seed_hi, realization;
    // soft source
    int src_on, src_comp, src_i, src_j, src_k;
    double src_amp, src_ws, src_tp, src_t0, dt;
    // loss box
    int box_on, box[6];
    // first-order Mur: one task per (axis a, side, component c)
    int n_mur;
    int mur_a[kMaxMurTasks], mur_side[kMaxMurTasks], mur_c[kMaxMurTasks];
    int bc[3];
    // graded lossy layer: loss per site = prof[x][hx][i] + prof[y][hy][j] + prof[z][hz][k]
    // (index 1 = half-integer position along that axis)
    int has_layer;
    const T* prof[3][2];
    // monitors
    Ctl* ctl;
    double* e_part;           // per workgroup energy partial sums
    double* l_part;           // per workgroup loss partial sums
    int n_part;
    double* hist;
    int64_t hist_cap;
    int n_probes, n_freq, decim;
    const int32_t* probe_comp;
    const int64_t* probe_off;
    T* ring;                  // n_probes x decim samples
    const double* omega;
    double* spec;             // n_probes x n_freq x 2
};

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, round
// multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /
// 0xBB67AE85.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t hi0 = __umulhi(0xD2511F53u, x0);
        const uint32_t lo0 = 0xD2511F53u * x0;
        const uint32_t hi1 = __umulhi(0xCD9E8D57u, x2);
        const uint32_t lo1 = 0xCD9E8D57u * x2;
        const uint32_t y0 = hi1 ^ x1 ^ k0;
        const uint32_t y2 = hi0 ^ x3 ^ k1;
        x0 = y0;
        x1 = lo1;
        x2 = y2;
        x3 = lo0;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
}

__device__ __forceinline__ void box_muller3(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                            float xi[3]) {
    // 24-bit uniforms (w >> 8 + 1/2) / 2^24: exact in binary32
    const float s = 5.9604644775390625e-8f;   // 2^-24
    const float u0 = ((float)(w0 >> 8) + 0.5f) * s;
    const float u1 = ((float)(w1 >> 8) + 0.5f) * s;
    const float u2 = ((float)(w2 >> 8) + 0.5f) * s;
    const float u3 = ((float)(w3 >> 8) + 0.5f) * s;
    const float r0 = sqrtf(-2.0f * logf(u0));
    const float r1 = sqrtf(-2.0f * logf(u2));
    float s1, c1, s3, c3;
    sincospif(2.0f * u1, &s1, &c1);
    sincospif(2.0f * u3, &s3, &c3);
    xi[0] = r0 * c1;
    xi[1] = r0 * s1;
    xi[2] = r1 * c3;
}

__device__ __forceinline__ void box_muller3(uint32_t w0, uint32_t w1, uint32_t w2, uint32_t w3,
                                            double xi[3]) {
    const double s = 5.9604644775390625e-8;
    const double u0 = ((double)(w0 >> 8) + 0.5) * s;
    const double u1 = ((double)(w1 >> 8) + 0.5) * s;
    const double u2 = ((double)(w2 >> 8) + 0.5) * s;
    const double u3 = ((double)(w3 >> 8) + 0.5) * s;
    const double r0 = sqrt(-2.0 * log(u0));
    const double r1 = sqrt(-2.0 * log(u2));
    double s1, c1, s3, c3;
    sincospi(2.0 * u1, &s1, &c1);
    sincospi(2.0 * u3, &s3, &c3);
    xi[0] = r0 * c1;
    xi[1] = r0 * s1;
    xi[2] = r1 * c3;
}

template <typename T>
__device__ __forceinline__ void noise3(const SimView<T>& v, uint32_t cell, uint32_t step,
                                       T xi[3]) {
    uint32_t x0 = cell, x1 = step, x2 = v.realization, x3 = 0u;
    philox4x32_10(x0, x1, x2, x3, v.seed_lo, v.seed_hi);
    box_muller3(x0, x1, x2, x3, xi);
}

// -------------------------------------------------------------- reductions
__device__ __forceinline__ double wave_sum(double x) {
#pragma unroll
    for (int o = 32; o > 0; o >>= 1) x += __shfl_xor(x, o, 64);
    return x;
}

// Sum over a workgroup of kThreads threads in a fixed order (deterministic).
__device__ __forceinline__ double block_sum(double x, double* sh) {
    const int t = threadIdx.x + threadIdx.y * blockDim.x;
    x = wave_sum(x);
    if ((t & 63) == 0) sh[t >> 6] = x;
    __syncthreads();
    double r = 0.0;
    if (t == 0) {
        const int nw = (blockDim.x * blockDim.y + 63) >> 6;
        for (int w = 0; w < nw; ++w) r += sh[w];
    }
    return r;
}

// Loss of an E-site of component c (half position along c) and of an H-site
// of component c (half positions along the two other axes).
template <typename T>
__device__ __forceinline__ T loss_e(const SimView<T>& v, int c, int i, int j, int k) {
    return (v.prof[0][c == 0][i] + v.prof[1][c == 1][j]) + v.prof[2][c == 2][k];
}
template <typename T>
__device__ __forceinline__ T loss_h(const SimView<T>& v, int c, int i, int j, int k) {
    return (v.prof[0][c != 0][i] + v.prof[1][c != 1][j]) + v.prof[2][c != 2][k];
}

// Faraday update with the semi-implicit loss of the layer
// (H' - H = -S curl - a (H' + H)); a = 0 is the plain Yee update.
template <typename T>
__device__ __forceinline__ T h_update(T h, T S, T curl, T a) {
    if (a == (T)0) return h - S * curl;
    const T ca = ((T)1 - a) / ((T)1 + a);
    const T cb = (T)1 / ((T)1 + a);
    return ca * h - cb * (S * curl);
}

template <typename T>
__device__ __forceinline__ T source_value(const SimView<T>& v, int64_t n) {
    const double t = (double)(n + 1) * v.dt - v.src_t0;
    const double q = t / v.src_tp;
    return (T)(v.src_amp * sin(v.src_ws * t) * exp(-q * q));
}

// ---------------------------------------------------------------- row a1
// H^{n+1/2} = H^{n-1/2} - S curl+ E^n on the H-sites of [0,n)^3, plus the
// energy W^n = 1/2 [sum eps E^n^2 (interior E-sites) + sum H^{n-1/2}.H^{n+1/2}
// (H-sites off the wall normal to their component)].
template <typename T>
__global__ void __launch_bounds__(kThreads) k_curl_h(SimView<T> v) {
    __shared__ double sh[kThreads / 64];
    const int i = blockIdx.x * kBlockX + threadIdx.x;
    const int j = blockIdx.y * kBlockY + threadIdx.y;
    const int k = blockIdx.z;
    const int64_t n = v.ctl->step;
    const int par = (int)(n & 1);
    double w = 0.0;
    if (i < v.nx && j < v.ny) {
        const T* __restrict__ Ex = v.E[par][0];
        const T* __restrict__ Ey = v.E[par][1];
        const T* __restrict__ Ez = v.E[par][2];
        const int64_t x = i + v.sx * j + v.sxy * k;
        const T ex = Ex[x], ey = Ey[x], ez = Ez[x];
        const T cx = (Ez[x + v.sx] - ez) - (Ey[x + v.sxy] - ey);
        const T cy = (Ex[x + v.sxy] - ex) - (Ez[x + 1] - ez);
        const T cz = (Ey[x + 1] - ey) - (Ex[x + v.sx] - ex);
        const T hx = v.H[par][0][x], hy = v.H[par][1][x], hz = v.H[par][2][x];
        T ax = (T)0, ay = (T)0, az = (T)0;
        if (v.has_layer) {
            ax = loss_h(v, 0, i, j, k);
            ay = loss_h(v, 1, i, j, k);
            az = loss_h(v, 2, i, j, k);
        }
        const T nhx = h_update(hx, v.S, cx, ax);
        const T nhy = h_update(hy, v.S, cy, ay);
        const T nhz = h_update(hz, v.S, cz, az);
        v.H[par ^ 1][0][x] = nhx;
        v.H[par ^ 1][1][x] = nhy;
        v.H[par ^ 1][2][x] = nhz;
        const T eps = v.lut_eps[v.mat[x]];
        T acc = (T)0;
        if (j >= 1 && k >= 1) acc += eps * ex * ex;
        if (i >= 1 && k >= 1) acc += eps * ey * ey;
        if (i >= 1 && j >= 1) acc += eps * ez * ez;
        if (i >= 1) acc += hx * nhx;
        if (j >= 1) acc += hy * nhy;
        if (k >= 1) acc += hz * nhz;
        w = 0.5 * (double)acc;
    }
    const double s = block_sum(w, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0)
        v.e_part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
}

// ---------------------------------------------------- rows a2, a3, a4, a5
template <typename T>
__device__ __forceinline__ void bloch_site(const SimView<T>& v, int c, int64_t x, T e, T curl,
                                           T ie, bool gain, T xi, T src, T* out_e, int par,
                                           T loss) {
    T dP = (T)0;
    T P = (T)0, Pn = (T)0;
    T n1 = (T)0, n2 = (T)0, n3 = (T)0;
    if (gain) {
        P = v.P[par][c][x];
        const T Pp = v.P[par ^ 1][c][x];
        n1 = v.N[0][c][x];
        n2 = v.N[1][c][x];
        n3 = v.N[2][c][x];
        Pn = v.a * P + v.b * Pp + v.ck * (n1 - n2) * e + v.cF * xi;
        dP = Pn - P;
    }
    T en;
    if (loss == (T)0) {
        en = e + ie * (v.S * curl - dP);
    } else {
        // semi-implicit loss of the layer: (E' - E) = (1/eps)(S curl - dP) - a (E' + E)
        const T ca = ((T)1 - loss) / ((T)1 + loss);
        const T cb = (T)1 / ((T)1 + loss);
        en = ca * e + cb * (ie * (v.S * curl - dP));
    }
    en += src;
    if (gain) {
        v.P[par ^ 1][c][x] = Pn;
        if (!v.frozen_pop) {
            const T W = v.beta * ((T)0.5 * (en + e)) * dP;
            const T n0 = v.Na - n1 - n2 - n3;
            v.N[2][c][x] = n3 + (v.dtWp * n0 - v.dt32 * n3);
            v.N[1][c][x] = n2 + (v.dt32 * n3 - v.dt21 * n2) + W;
            v.N[0][c][x] = n1 + (v.dt21 * n2 - v.dt10 * n1) - W;
        }
    }
    *out_e = en;
}

template <typename T>
__global__ void __launch_bounds__(kThreads) k_curl_e(SimView<T> v) {
    __shared__ double sh[kThreads / 64];
    const int i = blockIdx.x * kBlockX + threadIdx.x;
    const int j = blockIdx.y * kBlockY + threadIdx.y;
    const int k = blockIdx.z;
    const int64_t n = v.ctl->step;
    const int par = (int)(n & 1);
    double lsum = 0.0;
    if (i < v.nx && j < v.ny) {
        const int64_t x = i + v.sx * j + v.sxy * k;
        const T* __restrict__ Hx = v.H[par ^ 1][0];
        const T* __restrict__ Hy = v.H[par ^ 1][1];
        const T* __restrict__ Hz = v.H[par ^ 1][2];
        const uint8_t m = v.mat[x];
        const T ie = v.lut_inv_eps[m];
        const bool g = v.lut_gain[m] != 0;
        const bool inx = (j >= 1 && k >= 1), iny = (i >= 1 && k >= 1), inz = (i >= 1 && j >= 1);
        T xi[3] = {(T)0, (T)0, (T)0};
        if (g && v.noise && (inx || iny || inz)) {
            const uint32_t cell = (uint32_t)(i + v.nx * (j + v.ny * k));
            noise3(v, cell, (uint32_t)n, xi);
        }
        T srcv[3] = {(T)0, (T)0, (T)0};
        if (v.src_on && i == v.src_i && j == v.src_j && k == v.src_k) srcv[v.src_comp] = source_value(v, n);
        const bool inbox = v.box_on && i >= v.box[0] && i < v.box[3] && j >= v.box[1] &&
                           j < v.box[4] && k >= v.box[2] && k < v.box[5];
        T acc = (T)0;
        if (inx) {
            const T hz = Hz[x], hy = Hy[x];
            const T curl = (hz - Hz[x - v.sx]) - (hy - Hy[x - v.sxy]);
            T en;
            bloch_site(v, 0, x, v.E[par][0][x], curl, ie, g, xi[0], srcv[0], &en, par,
                       v.has_layer ? loss_e(v, 0, i, j, k) : (T)0);
            v.E[par ^ 1][0][x] = en;
            acc += en * en;
        }
        if (iny) {
            const T hx = Hx[x], hz = Hz[x];
            const T curl = (hx - Hx[x - v.sxy]) - (hz - Hz[x - 1]);
            T en;
            bloch_site(v, 1, x, v.E[par][1][x], curl, ie, g, xi[1], srcv[1], &en, par,
                       v.has_layer ? loss_e(v, 1, i, j, k) : (T)0);
            v.E[par ^ 1][1][x] = en;
            acc += en * en;
        }
        if (inz) {
            const T hy = Hy[x], hx = Hx[x];
            const T curl = (hy - Hy[x - 1]) - (hx - Hx[x - v.sx]);
            T en;
            bloch_site(v, 2, x, v.E[par][2][x], curl, ie, g, xi[2], srcv[2], &en, par,
                       v.has_layer ? loss_e(v, 2, i, j, k) : (T)0);
            v.E[par ^ 1][2][x] = en;
            acc += en * en;
        }
        if (inbox) lsum = (double)acc;
    }
    if (v.box_on) {
        const double s = block_sum(lsum, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0)
            v.l_part[blockIdx.x + gridDim.x * (blockIdx.y + gridDim.y * blockIdx.z)] = s;
    }
}

// ------------------------------------------------ fused step (a1 to a5)
// One workgroup owns a 64 x TY tile of (i, j) columns and marches along z over
// a segment [z0, z1) of planes.  Per plane k it stages E^n(k+1) (tile plus a
// one-site halo on every side) in LDS next to E^n(k), forms H^{n+1/2}(k) on the
// tile and on the low-side halo row and column that the E update needs, then
// updates E, P and the populations of the tile at plane k.  H^{n+1/2}(k-1) of
// its own columns stays in registers from the previous plane; a segment that
// does not start at z = 0 first recomputes plane z0-1 without storing it.
// Every value is formed by the same expression as in the two-pass kernels
// (k_curl_h, k_curl_e), so both paths give bitwise identical fields.
//
// Work items (tile x, tile y, segment) are laid out so that the workgroups
// that land on one XCD (the dispatcher deals workgroups round-robin over the
// 8 XCDs) get a contiguous run of neighbouring tiles and share halo lines in
// that XCD's L2.
struct FusedGeom {
    int tiles_x, tiles_y, segs, zseg, nblk, xcd_remap;
};

__device__ __forceinline__ int xcd_work_item(int b, int nblk, int remap) {
    if (!remap) return b;
    const int q = nblk >> 3, r = nblk & 7;
    const int x = b & 7, idx = b >> 3;
    return x * q + (x < r ? x : r) + idx;
}

template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY) k_step_fused(SimView<T> v, FusedGeom g) {
    constexpr int TX = 64;
    constexpr int LX = TX + 2, LY = TY + 2;      // E planes: x0-1 .. x0+64, y0-1 .. y0+TY
    constexpr int HX = TX + 1, HY = TY + 1;      // new H plane: x0-1 .. x0+63, y0-1 .. y0+TY-1
    __shared__ T se[2][3][LY][LX];
    __shared__ T sh[3][HY][HX];
    __shared__ double red[(64 * TY) / 64];
    const int w = xcd_work_item(blockIdx.x, g.nblk, g.xcd_remap);
    const int tx = threadIdx.x, ty = threadIdx.y;
    const int tid = tx + TX * ty;
    const int bx = w % g.tiles_x;
    const int by = (w / g.tiles_x) % g.tiles_y;
    const int bz = w / (g.tiles_x * g.tiles_y);
    const int x0 = bx * TX, y0 = by * TY;
    const int z0 = bz * g.zseg;
    const int z1 = min(z0 + g.zseg, v.nz);
    const int i = x0 + tx, j = y0 + ty;
    const bool act = i < v.nx && j < v.ny;
    const int64_t n = v.ctl->step;
    const int par = (int)(n & 1);
    const T* __restrict__ E0 = v.E[par][0];
    const T* __restrict__ E1 = v.E[par][1];
    const T* __restrict__ E2 = v.E[par][2];

    auto load_plane = [&](int buf, int k) {
        const int tot = 3 * LY * LX;
        for (int q = tid; q < tot; q += TX * TY) {
            const int c = q / (LY * LX);
            const int r = q % (LY * LX);
            const int ly = r / LX, lx = r % LX;
            const int gx = x0 - 1 + lx, gy = y0 - 1 + ly;
            T val = (T)0;
            if (k <= v.nz && gx >= 0 && gx <= v.nx && gy >= 0 && gy <= v.ny) {
                const int64_t x = gx + v.sx * gy + v.sxy * k;
                val = (c == 0 ? E0 : (c == 1 ? E1 : E2))[x];
            }
            se[buf][c][ly][lx] = val;
        }
    };

    double wsum = 0.0, lsum = 0.0;
    T hxp = (T)0, hyp = (T)0;
    const int kstart = z0 > 0 ? z0 - 1 : z0;
    int cur = 0;
    load_plane(cur, kstart);
    for (int k = kstart; k < z1; ++k) {
        const int nxt = cur ^ 1;
        load_plane(nxt, k + 1);
        __syncthreads();
        const bool own = k >= z0;
        // ---- a1: H^{n+1/2} at plane k
        T nhx = (T)0, nhy = (T)0, nhz = (T)0;
        const int ly = ty + 1, lx = tx + 1;
        if (act) {
            const int64_t x = i + v.sx * j + v.sxy * k;
            const T ex = se[cur][0][ly][lx], ey = se[cur][1][ly][lx], ez = se[cur][2][ly][lx];
            const T cx = (se[cur][2][ly + 1][lx] - ez) - (se[nxt][1][ly][lx] - ey);
            const T cy = (se[nxt][0][ly][lx] - ex) - (se[cur][2][ly][lx + 1] - ez);
            const T cz = (se[cur][1][ly][lx + 1] - ey) - (se[cur][0][ly + 1][lx] - ex);
            const T hx = v.H[par][0][x], hy = v.H[par][1][x], hz = v.H[par][2][x];
            T ax = (T)0, ay = (T)0, az = (T)0;
            if (v.has_layer) {
                ax = loss_h(v, 0, i, j, k);
                ay = loss_h(v, 1, i, j, k);
                az = loss_h(v, 2, i, j, k);
            }
            nhx = h_update(hx, v.S, cx, ax);
            nhy = h_update(hy, v.S, cy, ay);
            nhz = h_update(hz, v.S, cz, az);
            if (own) {
                v.H[par ^ 1][0][x] = nhx;
                v.H[par ^ 1][1][x] = nhy;
                v.H[par ^ 1][2][x] = nhz;
                const T eps = v.lut_eps[v.mat[x]];
                T acc = (T)0;
                if (j >= 1 && k >= 1) acc += eps * ex * ex;
                if (i >= 1 && k >= 1) acc += eps * ey * ey;
                if (i >= 1 && j >= 1) acc += eps * ez * ez;
                if (i >= 1) acc += hx * nhx;
                if (j >= 1) acc += hy * nhy;
                if (k >= 1) acc += hz * nhz;
                wsum += 0.5 * (double)acc;
            }
        }
        sh[0][ly][lx] = nhx;
        sh[1][ly][lx] = nhy;
        sh[2][ly][lx] = nhz;
        // low-side halo row (i, y0-1): Hx and Hz
        if (ty == 0 && y0 > 0 && i < v.nx) {
            const int64_t x = i + v.sx * (y0 - 1) + v.sxy * k;
            const T ex = se[cur][0][0][lx], ey = se[cur][1][0][lx], ez = se[cur][2][0][lx];
            const T cx = (se[cur][2][1][lx] - ez) - (se[nxt][1][0][lx] - ey);
            const T cz = (se[cur][1][0][lx + 1] - ey) - (se[cur][0][1][lx] - ex);
            const T ax = v.has_layer ? loss_h(v, 0, i, y0 - 1, k) : (T)0;
            const T az = v.has_layer ? loss_h(v, 2, i, y0 - 1, k) : (T)0;
            sh[0][0][lx] = h_update(v.H[par][0][x], v.S, cx, ax);
            sh[2][0][lx] = h_update(v.H[par][2][x], v.S, cz, az);
        }
        // low-side halo column (x0-1, j): Hy and Hz
        if (ty == 1 && tx < TY && x0 > 0 && y0 + tx < v.ny) {
            const int hj = y0 + tx;
            const int hly = tx + 1;
            const int64_t x = (x0 - 1) + v.sx * hj + v.sxy * k;
            const T ex = se[cur][0][hly][0], ey = se[cur][1][hly][0], ez = se[cur][2][hly][0];
            const T cy = (se[nxt][0][hly][0] - ex) - (se[cur][2][hly][1] - ez);
            const T cz = (se[cur][1][hly][1] - ey) - (se[cur][0][hly + 1][0] - ex);
            const T ay = v.has_layer ? loss_h(v, 1, x0 - 1, hj, k) : (T)0;
            const T az = v.has_layer ? loss_h(v, 2, x0 - 1, hj, k) : (T)0;
            sh[1][hly][0] = h_update(v.H[par][1][x], v.S, cy, ay);
            sh[2][hly][0] = h_update(v.H[par][2][x], v.S, cz, az);
        }
        __syncthreads();
        // ---- a2..a5 at plane k
        if (own && act) {
            const int64_t x = i + v.sx * j + v.sxy * k;
            const uint8_t m = v.mat[x];
            const T ie = v.lut_inv_eps[m];
            const bool gn = v.lut_gain[m] != 0;
            const bool inx = (j >= 1 && k >= 1), iny = (i >= 1 && k >= 1), inz = (i >= 1 && j >= 1);
            T xi[3] = {(T)0, (T)0, (T)0};
            if (gn && v.noise && (inx || iny || inz)) {
                const uint32_t cell = (uint32_t)(i + v.nx * (j + v.ny * k));
                noise3(v, cell, (uint32_t)n, xi);
            }
            T srcv[3] = {(T)0, (T)0, (T)0};
            if (v.src_on && i == v.src_i && j == v.src_j && k == v.src_k)
                srcv[v.src_comp] = source_value(v, n);
            T acc = (T)0;
            if (inx) {
                const T curl = (sh[2][ly][lx] - sh[2][ly - 1][lx]) - (sh[1][ly][lx] - hyp);
                T en;
                bloch_site(v, 0, x, se[cur][0][ly][lx], curl, ie, gn, xi[0], srcv[0], &en, par,
                           v.has_layer ? loss_e(v, 0, i, j, k) : (T)0);
                v.E[par ^ 1][0][x] = en;
                acc += en * en;
            }
            if (iny) {
                const T curl = (sh[0][ly][lx] - hxp) - (sh[2][ly][lx] - sh[2][ly][lx - 1]);
                T en;
                bloch_site(v, 1, x, se[cur][1][ly][lx], curl, ie, gn, xi[1], srcv[1], &en, par,
                           v.has_layer ? loss_e(v, 1, i, j, k) : (T)0);
                v.E[par ^ 1][1][x] = en;
                acc += en * en;
            }
            if (inz) {
                const T curl = (sh[1][ly][lx] - sh[1][ly][lx - 1]) - (sh[0][ly][lx] - sh[0][ly - 1][lx]);
                T en;
                bloch_site(v, 2, x, se[cur][2][ly][lx], curl, ie, gn, xi[2], srcv[2], &en, par,
                           v.has_layer ? loss_e(v, 2, i, j, k) : (T)0);
                v.E[par ^ 1][2][x] = en;
                acc += en * en;
            }
            if (v.box_on && i >= v.box[0] && i < v.box[3] && j >= v.box[1] && j < v.box[4] &&
                k >= v.box[2] && k < v.box[5])
                lsum += (double)acc;
        }
        hxp = nhx;
        hyp = nhy;
        __syncthreads();
        cur = nxt;
    }
    const double ws = block_sum(wsum, red);
    __syncthreads();
    const double ls = v.box_on ? block_sum(lsum, red) : 0.0;
    if (tid == 0) {
        v.e_part[blockIdx.x] = ws;
        if (v.box_on) v.l_part[blockIdx.x] = ls;
    }
}

// ---------------------------------------------------------------- row a6
// First-order Mur on the wall E-sites of Mur axes.  Task (a, side, c) covers
// the sites of component c on the wall i_a = 0 or n_a.  A site that also lies
// on the wall of the third axis t belongs to the face applied last in x, y, z
// order; when that is face a (t < a) the neighbour it reads is itself a
// face-t site, whose new value is formed inline.  Sites on PEC walls stay 0.
template <typename T>
__global__ void __launch_bounds__(256) k_mur(SimView<T> v) {
    const int task = blockIdx.y;
    const int a = v.mur_a[task], side = v.mur_side[task], c = v.mur_c[task];
    const int t = 3 - a - c;
    const int nd[3] = {v.nx, v.ny, v.nz};
    const int nc = nd[c], nt = nd[t] + 1;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)nc * nt) return;
    const int u = (int)(q % nc);
    const int w = (int)(q / nc);
    const bool on_t = (w == 0 || w == nd[t]);
    if (on_t && (v.bc[t] != 1 || t > a)) return;
    const int64_t par = v.ctl->step & 1;   // parity of the step being finished
    const T* __restrict__ Ec = v.E[par][c];
    T* __restrict__ En = v.E[par ^ 1][c];
    const int64_t st[3] = {1, v.sx, v.sxy};
    const int wall = side ? nd[a] : 0;
    const int inner = side ? nd[a] - 1 : 1;
    const int64_t s = (int64_t)wall * st[a] + (int64_t)u * st[c] + (int64_t)w * st[t];
    const int64_t s1 = s + (int64_t)(inner - wall) * st[a];
    T e1new;
    if (!on_t) {
        e1new = En[s1];
    } else {
        const int tin = (w == 0) ? 1 : nd[t] - 1;
        const int64_t s2 = s1 + (int64_t)(tin - w) * st[t];
        const T m1 = v.lut_mur[v.mat[s1]];
        e1new = Ec[s2] + m1 * (En[s2] - Ec[s1]);
    }
    const T m = v.lut_mur[v.mat[s]];
    En[s] = Ec[s1] + m * (e1new - Ec[s]);
}

// ------------------------------------------------------ row a7, step end
template <typename T>
__global__ void __launch_bounds__(256) k_end_step(SimView<T> v) {
    __shared__ double sh[4];
    const int t = threadIdx.x;
    const int64_t n = v.ctl->step;
    double acc = 0.0;
    for (int q = t; q < v.n_part; q += 256) acc += v.e_part[q];
    // fixed-order tree over the 256 strided partial sums
    double W = wave_sum(acc);
    if ((t & 63) == 0) sh[t >> 6] = W;
    __syncthreads();
    W = sh[0] + sh[1] + sh[2] + sh[3];
    __syncthreads();
    double L = 0.0;
    if (v.box_on) {
        double la = 0.0;
        for (int q = t; q < v.n_part; q += 256) la += v.l_part[q];
        la = wave_sum(la);
        if ((t & 63) == 0) sh[t >> 6] = la;
        __syncthreads();
        L = sh[0] + sh[1] + sh[2] + sh[3];
    }
    const int par1 = (int)((n + 1) & 1);
    for (int p = t; p < v.n_probes; p += 256)
        v.ring[(int64_t)p * v.decim + (n % v.decim)] = v.E[par1][v.probe_comp[p]][v.probe_off[p]];
    if (t == 0) {
        if (!(W == W) || W - W != 0.0) v.ctl->nonfinite = 1;
        if (n < v.hist_cap) v.hist[n] = W;
        v.ctl->W_now = W;
        v.ctl->W_int += W;
        v.ctl->loss += L;
        v.ctl->step = n + 1;
    }
}

// Fold `count` buffered probe samples into the FP64 spectrum; the samples
// are m = step-count+1 .. step (E^m), stored at ring slot (m-1) mod decim.
template <typename T>
__global__ void __launch_bounds__(256) k_dft(SimView<T> v, int count) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)v.n_probes * v.n_freq) return;
    const int p = (int)(q / v.n_freq);
    const int f = (int)(q % v.n_freq);
    const int64_t m0 = v.ctl->step - count + 1;
    const double w = v.omega[f] * v.dt;
    double re = 0.0, im = 0.0;
    for (int r = 0; r < count; ++r) {
        const int64_t m = m0 + r;
        const double e = (double)v.ring[(int64_t)p * v.decim + ((m - 1) % v.decim)];
        double sn, cs;
        sincos(w * (double)m, &sn, &cs);
        re += e * cs;
        im += e * sn;
    }
    v.spec[2 * q] += re;
    v.spec[2 * q + 1] += im;
}

// ------------------------------------------------------------ set-up
// Populations of every interior gain E-site at their initial values.
template <typename T>
__global__ void __launch_bounds__(256) k_init_pop(SimView<T> v, T n1, T n2, T n3) {
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    const int64_t tot = v.sxy * (int64_t)(v.nz + 1);
    if (q >= tot) return;
    const int k = (int)(q / v.sxy);
    const int64_t r = q % v.sxy;
    const int j = (int)(r / v.sx);
    const int i = (int)(r % v.sx);
    const bool cellok = i < v.nx && j < v.ny && k < v.nz && v.lut_gain[v.mat[q]];
    const bool in[3] = {cellok && j >= 1 && k >= 1, cellok && i >= 1 && k >= 1,
                        cellok && i >= 1 && j >= 1};
    for (int c = 0; c < 3; ++c) {
        v.N[0][c][q] = in[c] ? n1 : (T)0;
        v.N[1][c][q] = in[c] ? n2 : (T)0;
        v.N[2][c][q] = in[c] ? n3 : (T)0;
    }
}

}  // namespace mbf
