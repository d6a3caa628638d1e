// Device code of the Maxwell-Bloch FDTD step for gfx950 (wave64).
//
// Layout: every E and H component is a structure-of-arrays array over the
// extended Yee index range (nx+1)*(ny+1)*(nz+1), x fastest, rows padded to
// 128-byte lines.  E and H are double-buffered (the step reads buffer `par`
// and writes buffer `par^1`, par = step & 1), so a kernel never reads a value
// another workgroup of the same launch may already have overwritten.
//
// The Bloch state (P^n, P^{n-1}, N1..N3 per component) exists only on gain
// cells and is stored compactly, one value per gain cell in every component
// array.  The cells are cut into 64-wide x segments of one row and plane,
// numbered in memory order (bx + nbx (j + ny k)), and the gain cells in that
// order.  A cell's number is the count of gain cells before its segment (a
// table with one entry per segment) plus the number of gain lanes below it in
// the wave that covers the segment (a ballot and a bit count), so the Bloch
// loads and stores of a wave touch consecutive addresses, every cache line
// carries gain sites only, and the workgroups that run together (neighbours in
// x and y) stream through one region of every array.  P^{n+1} is written over
// P^{n-1}; N1..N3 are updated in place.  Material is one byte per site: an
// index into a small table of (1/eps_r, eps_r, Mur coefficient); ids from
// kGainId up mark gain cells, so the gain flag needs no table look-up.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace mbf {

constexpr int kMaxMat = 256;
constexpr int kGainId = 128;  // material ids >= kGainId are gain cells
constexpr int kMaxMurTasks = 12;

struct Ctl {                  // per-simulation control block (device memory)
    int64_t step;             // steps taken since the pump was set
    double W_now;             // energy of the last step
    double W_int;             // sum of the energy over all steps
    double loss;              // loss-box integral
    int32_t nonfinite;        // set once a step produced a non-finite energy
    int32_t pad;
    double src_val;           // soft-source value added during the current step
    int64_t tap_base;         // step of trajectory slot 0 while a trajectory is recorded
};

template <typename T>
struct SimView {
    using value_type = T;
    T* E[2][3];
    T* H[2][3];
    T* P[2][3];               // compact, one value per gain cell
    T* N[3][3];               // N1, N2, N3 x component, compact
    const uint32_t* seg_base; // gain cells before segment (bx, j, k), bx + nbx (j + ny k)
    // trajectory recording for the adjoint (tap == nullptr: off): the E pass
    // writes E^{n+1}, P^{n+1} - P^n and N1 - N2 at n+1 into slot
    // n + 1 - ctl->tap_base of tap_stride values: E (3 x tap_e dense), dP
    // (3 x tap_c compact), N1 - N2 (3 x tap_c compact)
    T* tap;
    int64_t tap_stride, tap_e, tap_c;
    int nbx;                  // 64-wide segments per row
    const uint8_t* mat;       // per site of the extended range
    const T* lut_inv_eps;     // per material id
    const T* lut_eps;
    const T* lut_mur;
    int nx, ny, nz;
    int64_t sx, sxy;          // strides of the extended range
    T S, a, b, ck, cF, beta, dt32, dt21, dt10, dtWp, Na;
    int noise;
    int frozen_pop;
    uint32_t seed_lo, seed_hi, realization;
    // soft source: src_kind 0 is the Gaussian pulse (src_tp its width, src_t0
    // its centre), 1 the continuous wave switched on over src_tp
    int src_on, src_kind, src_comp, src_i, src_j, src_k;
    double src_amp, src_ws, src_tp, src_t0, dt;
    // loss box
    int box_on, box[6];
    // first-order Mur: task q (a, side, c) packed in bits 5q..5q+4 of mur_code
    // as a | side << 2 | c << 3; bit a of mur_axes set when axis a is Mur
    int n_mur;
    uint64_t mur_code;
    int mur_axes;
    // graded lossy layer: the coefficients (ca, cb) of a site's semi-implicit
    // update are the pair at entry lev[0][hx][i] * lc_sy + lev[1][hy][j] *
    // lc_sz + lev[2][hz][k] of lc, where lev[a][h][q] numbers the distinct
    // profile values of axis a (h = 1: half-integer position; level 0 is the
    // value 0, so entry 0 is (1, 1) and stands for a site outside the layer)
    int has_layer;
    const uint8_t* lev[3][2];
    const T* lc;
    uint32_t lc_sy, lc_sz;
    int lay_kz[2];            // planes lay_kz[0] <= k < lay_kz[1] have zero z parts
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
    // energy density of the cells of plane z = map_k summed over steps
    // (nx x ny, x fastest; map == nullptr: off)
    double* map;
    int map_k;
};

// ------------------------------------------------------------------ Philox
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11): ten rounds, round
// multipliers 0xD2511F53 / 0xCD9E8D57, Weyl key increments 0x9E3779B9 /
// 0xBB67AE85.
__device__ __forceinline__ void philox4x32_10(uint32_t& x0, uint32_t& x1, uint32_t& x2,
                                              uint32_t& x3, uint32_t k0, uint32_t k1) {
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint64_t p0 = (uint64_t)0xD2511F53u * x0;   // one v_mad_u64_u32 each
        const uint64_t p1 = (uint64_t)0xCD9E8D57u * x2;
        const uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        const uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
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
    // hardware transcendentals: log2, square root, and sin/cos of 2*pi*u
    // (the sin/cos units take their argument in revolutions); u lies in (0,1)
    const float ln2x2 = 1.3862943611198906f;     // 2 ln 2
    const float r0 = __builtin_amdgcn_sqrtf(-ln2x2 * __builtin_amdgcn_logf(u0));
    const float r1 = __builtin_amdgcn_sqrtf(-ln2x2 * __builtin_amdgcn_logf(u2));
    xi[0] = r0 * __builtin_amdgcn_cosf(u1);
    xi[1] = r0 * __builtin_amdgcn_sinf(u1);
    xi[2] = r1 * __builtin_amdgcn_cosf(u3);
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
    const double c1 = cospi(2.0 * u1), s1 = sinpi(2.0 * u1);
    const double c3 = cospi(2.0 * u3);
    xi[0] = r0 * c1;
    xi[1] = r0 * s1;
    xi[2] = r1 * c3;
}

template <typename V, typename T>
__device__ __forceinline__ void noise3(const V& v, uint32_t cell, uint32_t step, T xi[3]) {
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

// Sum over a workgroup in a fixed order (deterministic); thread 0 gets the sum.
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

// Loads and stores at a 32-bit element offset from a uniform base: the
// address is base + zero-extended 32-bit byte offset, which maps to the
// scalar-base form of the global memory instructions.  The pointers are
// cast to the global address space: a pointer read from a view in memory
// (the batched kernels) would otherwise be generic and use flat accesses.
#define MBF_GLOBAL __attribute__((address_space(1)))
template <typename T>
__device__ __forceinline__ T ldo(const T* base, uint32_t off) {
    const MBF_GLOBAL char* b = (const MBF_GLOBAL char*)base;
    return *(const MBF_GLOBAL T*)(b + off * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void sto(T* base, uint32_t off, T val) {
    MBF_GLOBAL char* b = (MBF_GLOBAL char*)base;
    *(MBF_GLOBAL T*)(b + off * (uint32_t)sizeof(T)) = val;
}
// Streaming store (non-temporal: the line is not kept in the caches).
template <typename T>
__device__ __forceinline__ void sto_nt(T* base, uint32_t off, T val) {
    MBF_GLOBAL char* b = (MBF_GLOBAL char*)base;
    __builtin_nontemporal_store(val, (MBF_GLOBAL T*)(b + off * (uint32_t)sizeof(T)));
}
template <typename T>
__device__ __forceinline__ T gld(const T* p) {
    return *(const MBF_GLOBAL T*)p;
}

// Field pointers of one step, chosen once per kernel from the step parity
// (uniform selects; the kernel-argument arrays are only ever indexed with
// compile-time constants, so nothing is copied to private memory).
template <typename T>
struct Fields {
    const T* e[3];    // E^n
    T* en[3];         // E^{n+1}
    const T* h[3];    // H^{n-1/2}
    T* hn[3];         // H^{n+1/2}
    const T* p[3];    // P^n
    T* q[3];          // P^{n-1} on entry, P^{n+1} on exit
    T* n1[3];
    T* n2[3];
    T* n3[3];
};

template <typename T>
__device__ __forceinline__ Fields<T> bind_fields(const SimView<T>& v, int par) {
    Fields<T> f;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        f.e[c] = par ? v.E[1][c] : v.E[0][c];
        f.en[c] = par ? v.E[0][c] : v.E[1][c];
        f.h[c] = par ? v.H[1][c] : v.H[0][c];
        f.hn[c] = par ? v.H[0][c] : v.H[1][c];
        f.p[c] = par ? v.P[1][c] : v.P[0][c];
        f.q[c] = par ? v.P[0][c] : v.P[1][c];
        f.n1[c] = v.N[0][c];
        f.n2[c] = v.N[1][c];
        f.n3[c] = v.N[2][c];
    }
    return f;
}

// Layer coefficients of a site: ca = (1 - a)/(1 + a) and cb = 1/(1 + a) for
// its summed loss a, formed on the host in FP64 and rounded once to the field
// type, like every other coefficient.  (1, 1) outside the layer, where the
// semi-implicit updates reduce to the plain Yee ones bit for bit (1 * x == x).
template <typename T>
struct LayC {
    T ca, cb;
};

// Table entry of a site from the parts of its three axes (lev * stride).
template <typename T>
__device__ __forceinline__ LayC<T> lay_coef(const T* lc, uint32_t t) {
    LayC<T> r{(T)1, (T)1};
    if (t != 0u) {
        r.ca = ldo(lc, 2u * t);
        r.cb = ldo(lc, 2u * t + 1u);
    }
    return r;
}

// Per-axis parts of the table entry: axis a at index q, integer (hf = 0) or
// half-integer (hf = 1) position.
template <typename V>
__device__ __forceinline__ uint32_t lay_part(const V& v, int a, int hf, int q) {
    const uint32_t l = gld(v.lev[a][hf] + q);
    return a == 0 ? l * v.lc_sy : (a == 1 ? l * v.lc_sz : l);
}

// Entry of an E-site of component c (half position along c) and of an H-site
// of component c (half positions along the two other axes).
template <typename V>
__device__ __forceinline__ LayC<typename V::value_type> lay_coef_e(const V& v, int c, int i, int j, int k) {
    if (!v.has_layer) return {(typename V::value_type)1, (typename V::value_type)1};
    return lay_coef(v.lc, lay_part(v, 0, c == 0, i) + lay_part(v, 1, c == 1, j) + lay_part(v, 2, c == 2, k));
}
template <typename V>
__device__ __forceinline__ LayC<typename V::value_type> lay_coef_h(const V& v, int c, int i, int j, int k) {
    if (!v.has_layer) return {(typename V::value_type)1, (typename V::value_type)1};
    return lay_coef(v.lc, lay_part(v, 0, c != 0, i) + lay_part(v, 1, c != 1, j) + lay_part(v, 2, c != 2, k));
}

// Compact index of the calling lane's cell in the Bloch-state arrays.  Must
// be called by the whole wave that covers x segment bx of row (j, k) (lanes
// outside the grid inactive or with g = false); j and k are wave-uniform and
// row_ok is false for a wave past the last row (its result is then unused).
template <typename V>
__device__ __forceinline__ uint32_t gain_index(const V& v, int bx, int j, int k, bool g, bool row_ok) {
    const uint64_t mask = __ballot(g);
    const uint32_t below = __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                                     __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
    const int seg = __builtin_amdgcn_readfirstlane(bx + v.nbx * (j + v.ny * k));
    const uint32_t base = row_ok ? gld(v.seg_base + seg) : 0u;
    return base + below;
}

// Curl component from two differences of neighbours: (a - b) - (c - d).
template <typename T>
__device__ __forceinline__ T dcurl(T a, T b, T c, T d) {
    return (a - b) - (c - d);
}

// Faraday update with the semi-implicit loss of the layer
// (H' - H = -S curl - a (H' + H)); ca = cb = 1 is the plain Yee update.
template <typename T>
__device__ __forceinline__ T h_update(T h, T S, T curl, LayC<T> l) {
    return l.ca * h - l.cb * (S * curl);
}

template <typename V>
__device__ __forceinline__ double source_at(const V& v, int64_t n) {
    if (v.src_kind == 1) {
        const double t = (double)(n + 1) * v.dt;
        const double q = t / v.src_tp;
        return v.src_amp * (1.0 - exp(-q * q)) * sin(v.src_ws * t);
    }
    const double t = (double)(n + 1) * v.dt - v.src_t0;
    const double q = t / v.src_tp;
    return v.src_amp * sin(v.src_ws * t) * exp(-q * q);
}

template <typename T>
__device__ __forceinline__ T source_value(const SimView<T>& v, int64_t n) {
    return (T)source_at(v, n);
}

// Work decomposition of the step kernels: tiles of 64 x TY columns cut into
// z segments of zseg planes, one workgroup each, on a 1-D grid of nblk.
struct Geom {
    int tiles_x, tiles_y, segs, zseg, nblk, xcd_remap;
};

// Workgroups are dealt to the 8 XCDs in turn (id mod 8); with remapping, XCD
// x takes the x-th contiguous range of work items instead, so neighbouring
// items (the next tile in x or y, whose halo rows and Bloch-array lines they
// share) meet in the same L2.  The reverse-step kernels map their workgroups
// this way; the step kernels read a work table the host writes in dispatch
// order.
__device__ __forceinline__ int xcd_work_item(int b, int nblk, int remap) {
    if (!remap) return b;
    remap = 1;
    const int q = nblk >> 3, r = nblk & 7;
    const int x = b & 7, idx = b >> 3;
    return x * q + (x < r ? x : r) + idx;
}

// Work item -> (x tile, y tile, z segment), x tile fastest (memory order).
__device__ __forceinline__ void decode_item(const Geom& g, int w, int& bx, int& by, int& bz) {
    bx = w % g.tiles_x;
    const int r = w / g.tiles_x;
    by = r % g.tiles_y;
    bz = r / g.tiles_y;
}

// A batch of simulations stepped by one launch per kernel: the device array
// of the members' views and geometries, and a work table whose entry q holds
// (member << 24) | work item for workgroup q of the launch (the host lays the
// table out in dispatch order, XCD grouping included).  Energy and loss partials are indexed by the member's own
// work item, so a member's sums match its solo run term for term.

__device__ __forceinline__ void batch_item(const uint32_t* __restrict__ items, int nitems, int remap,
                                           int& r, int& w) {
    (void)nitems;
    (void)remap;                       // the table is already in dispatch order
    const uint32_t e = items[blockIdx.x];
    r = (int)(e >> 24);
    w = (int)(e & 0xFFFFFFu);
}

// Energy density of cell (i, j) of the monitored plane from the cell's own
// sites, 1/2 [eps_r |E^n|^2 + |H^{n+1/2}|^2], added to its FP64 sum (one lane
// owns each cell of the plane).
template <typename T>
__device__ __forceinline__ void plane_energy(const SimView<T>& v, int i, int j, T eps, T ex, T ey, T ez,
                                             T hx, T hy, T hz) {
    const double e2 = ((double)ex * (double)ex + (double)ey * (double)ey) + (double)ez * (double)ez;
    const double h2 = ((double)hx * (double)hx + (double)hy * (double)hy) + (double)hz * (double)hz;
    const uint32_t c = (uint32_t)i + (uint32_t)v.nx * (uint32_t)j;
    sto(v.map, c, gld(v.map + c) + 0.5 * ((double)eps * e2 + h2));
}

// ---------------------------------------------------------------- row a1
// H^{n+1/2} = H^{n-1/2} - S curl+ E^n on the H-sites of [0,n)^3, plus the
// energy W^n = 1/2 [sum eps E^n^2 (interior E-sites) + sum H^{n-1/2}.H^{n+1/2}
// (H-sites off the wall normal to their component)].
// Everything the H pass reads for one plane of a row: E^n at the site and at
// its +x, +y, +z neighbours, H^{n-1/2} and the material byte.
template <typename T>
struct HPlane {
    T ez, exk, eyk, ezy, ezx, eyx, exy, hx, hy, hz;
    uint8_t m;
};

template <typename T>
__device__ __forceinline__ void load_hplane(HPlane<T>& p, const Fields<T>& f, const uint8_t* mat, uint32_t x,
                                            uint32_t sx, uint32_t sxy) {
    p.ez = ldo(f.e[2], x);
    p.exk = ldo(f.e[0], x + sxy);
    p.eyk = ldo(f.e[1], x + sxy);
    p.ezy = ldo(f.e[2], x + sx);
    p.ezx = ldo(f.e[2], x + 1u);
    p.eyx = ldo(f.e[1], x + 1u);
    p.exy = ldo(f.e[0], x + sx);
    p.hx = ldo(f.h[0], x);
    p.hy = ldo(f.h[1], x);
    p.hz = ldo(f.h[2], x);
    p.m = ldo(mat, x);
}

// NT: H^{n+1/2} leaves by streaming stores (for grids far larger than the
// caches, where the E pass reads it back from HBM anyway).
template <typename T, int TY, bool NT>
__device__ __forceinline__ void curl_h_body(const SimView<T>& v, const Geom& gm, int w) {
    __shared__ double sh[TY];
    int bx, by, bz;
    decode_item(gm, w, bx, by, bz);
    const int i = bx * 64 + threadIdx.x;
    const int j = by * TY + threadIdx.y;
    const int64_t n = gld(&v.ctl->step);
    const int par = (int)(n & 1);
    const Fields<T> f = bind_fields(v, par);
    T wsum = (T)0;
    const int kz0 = bz * gm.zseg, kz1 = min(kz0 + gm.zseg, v.nz);
    if (i < v.nx && j < v.ny) {
        const T* __restrict__ Ex = f.e[0];
        const T* __restrict__ Ey = f.e[1];
        const uint32_t sx = (uint32_t)v.sx, sxy = (uint32_t)v.sxy;
        uint32_t x = (uint32_t)i + sx * (uint32_t)j + sxy * (uint32_t)kz0;
        // E^n at plane k is carried from the previous plane's k+1 loads; the
        // next plane's loads go out before this plane's arithmetic and stores
        // (all offsets are +1 along x, y or z: at most column nx, row ny,
        // plane nz of the extended range)
        T ex = ldo(Ex, x), ey = ldo(Ey, x);
        // the x and y parts of the sites' layer-table entries stay fixed along
        // the march in z (lay_coef_h: Hx at the integer x position and half
        // y, z positions, and so on; the row j is wave-uniform)
        uint32_t txy0 = 0u, txy1 = 0u, txy2 = 0u;
        if (v.has_layer) {
            const uint32_t tx0 = lay_part(v, 0, 0, i), tx1 = lay_part(v, 0, 1, i);
            const int jw = __builtin_amdgcn_readfirstlane(j);
            const uint32_t ty0 = lay_part(v, 1, 0, jw), ty1 = lay_part(v, 1, 1, jw);
            txy0 = tx0 + ty1;
            txy1 = tx1 + ty0;
            txy2 = tx1 + ty1;
        }
        const LayC<T> hx0 = lay_coef(v.lc, txy0), hy0 = lay_coef(v.lc, txy1), hz0 = lay_coef(v.lc, txy2);
        HPlane<T> P, Q;
        load_hplane(P, f, v.mat, x, sx, sxy);
        for (int k = kz0; k < kz1; ++k, x += sxy) {
            if (k + 1 < kz1) load_hplane(Q, f, v.mat, x + sxy, sx, sxy);
            const T ez = P.ez;
            const T exk = P.exk, eyk = P.eyk;
            const T cx = dcurl(P.ezy, ez, eyk, ey);
            const T cy = dcurl(exk, ex, P.ezx, ez);
            const T cz = dcurl(P.eyx, ey, P.exy, ex);
            const T hx = P.hx, hy = P.hy, hz = P.hz;
            // planes outside the z layer (all but 2L of them) use the
            // column's coefficients taken before the march
            uint32_t tz0 = 0u, tz1 = 0u;
            if (v.has_layer && (k < v.lay_kz[0] || k >= v.lay_kz[1])) {
                tz0 = lay_part(v, 2, 0, k);
                tz1 = lay_part(v, 2, 1, k);
            }
            LayC<T> ax = hx0, ay = hy0, az = hz0;
            if (tz0 | tz1) {
                ax = lay_coef(v.lc, txy0 + tz1);
                ay = lay_coef(v.lc, txy1 + tz1);
                az = lay_coef(v.lc, txy2 + tz0);
            }
            const T nhx = h_update(hx, v.S, cx, ax);
            const T nhy = h_update(hy, v.S, cy, ay);
            const T nhz = h_update(hz, v.S, cz, az);
            if constexpr (NT) {
                sto_nt(f.hn[0], x, nhx);
                sto_nt(f.hn[1], x, nhy);
                sto_nt(f.hn[2], x, nhz);
            } else {
                sto(f.hn[0], x, nhx);
                sto(f.hn[1], x, nhy);
                sto(f.hn[2], x, nhz);
            }
            const T eps = gld(v.lut_eps + P.m);
            if (v.map != nullptr && k == v.map_k) plane_energy(v, i, j, eps, ex, ey, ez, nhx, nhy, nhz);
            T acc = (T)0;
            if (j >= 1 && k >= 1) acc += eps * ex * ex;
            if (i >= 1 && k >= 1) acc += eps * ey * ey;
            if (i >= 1 && j >= 1) acc += eps * ez * ez;
            if (i >= 1) acc += hx * nhx;
            if (j >= 1) acc += hy * nhy;
            if (k >= 1) acc += hz * nhz;
            wsum += (T)0.5 * acc;
            ex = exk;
            ey = eyk;
            P = Q;
        }
    }
    const double s = block_sum((double)wsum, sh);
    if (threadIdx.x == 0 && threadIdx.y == 0) sto(v.e_part, (uint32_t)w, s);
}

// The tables are separate no-alias read-only arguments, so the compiler may
// keep the member's view in scalar registers across the kernel's stores.
template <typename T, int TY, bool NT>
__global__ void __launch_bounds__(64 * TY) k_curl_h_batch(const SimView<T>* __restrict__ views,
                                                const Geom* __restrict__ geoms,
                                                const uint32_t* __restrict__ items, int nitems, int remap) {
    int r, w;
    batch_item(items, nitems, remap, r, w);
    curl_h_body<T, TY, NT>(views[r], geoms[r], w);
}

// ---------------------------------------------------- rows a2, a3, a4, a5
// Per-site Bloch state of one E-site: P^n, P^{n-1} and N1..N3 (zero where
// the site carries no gain).  Loaded ahead of the update so that the loads are
// in flight while the field part of the step is computed.
template <typename T>
struct BlochIn {
    T P, Pp, n1, n2, n3;
};

template <typename T>
__device__ __forceinline__ BlochIn<T> bloch_load(const Fields<T>& f, int c, uint32_t gi, bool gain) {
    BlochIn<T> b{(T)0, (T)0, (T)0, (T)0, (T)0};
    if (gain) {
        b.P = ldo(f.p[c], gi);
        b.Pp = ldo(f.q[c], gi);
        b.n1 = ldo(f.n1[c], gi);
        b.n2 = ldo(f.n2[c], gi);
        b.n3 = ldo(f.n3[c], gi);
    }
    return b;
}

// Rows a2-a5 at one E-site from its loaded Bloch state.  `upd` marks an
// interior site (updated by Ampere's law; other sites keep E), `gain` an
// interior site of a gain cell, gi the cell's compact index.  Returns E^{n+1}.
template <typename T>
__device__ __forceinline__ T bloch_site(const SimView<T>& v, const Fields<T>& f, int c, uint32_t gi,
                                        T e, T curl, T ie, bool upd, bool gain,
                                        const BlochIn<T>& b, T xi, T src, LayC<T> lay, T* tslot) {
    T dP = (T)0;
    T Pn = (T)0;
    if (gain) {
        Pn = v.a * b.P + v.b * b.Pp + v.ck * (b.n1 - b.n2) * e + v.cF * xi;
        dP = Pn - b.P;
    }
    // semi-implicit loss of the layer: (E' - E) = (1/eps)(S curl - dP) - a (E' + E)
    T en = lay.ca * e + lay.cb * (ie * (v.S * curl - dP));
    en += src;
    en = upd ? en : e;
    if (gain) {
        sto(f.q[c], gi, Pn);
        T d12 = b.n1 - b.n2;
        if (!v.frozen_pop) {
            const T n1 = b.n1, n2 = b.n2, n3 = b.n3;
            const T W = v.beta * ((T)0.5 * (en + e)) * dP;
            // N0 = N_a - N1 - N2 - N3, with N_a - N2 taken first: N2 holds
            // nearly all atoms of a pumped site, that difference of nearly
            // equal values is exact, and N0 keeps its full precision (taking
            // N1 from N_a first would round at the scale of N_a, a relative
            // error of order 1e-4 in N0, whose pump term sets N3's fixed point)
            const T n0 = (v.Na - n2) - (n1 + n3);
            const T m2 = n2 + (v.dt32 * n3 - v.dt21 * n2) + W;
            const T m1 = n1 + (v.dt21 * n2 - v.dt10 * n1) - W;
            sto(f.n3[c], gi, n3 + (v.dtWp * n0 - v.dt32 * n3));
            sto(f.n2[c], gi, m2);
            sto(f.n1[c], gi, m1);
            d12 = m1 - m2;
        }
        if (tslot) {
            sto(tslot + 3 * v.tap_e + c * v.tap_c, gi, dP);
            sto(tslot + 3 * v.tap_e + 3 * v.tap_c + c * v.tap_c, gi, d12);
        }
    }
    return en;
}

// Base of the trajectory slot that step n writes (nullptr when not recording).
template <typename T>
__device__ __forceinline__ T* tap_slot(const SimView<T>& v, int64_t n) {
    return v.tap ? v.tap + (n + 1 - gld(&v.ctl->tap_base)) * v.tap_stride : nullptr;
}

// The soft source's value for component c at this site (zero elsewhere).
template <typename T>
__device__ __forceinline__ void source3(const SimView<T>& v, int i, int j, int k, int64_t n,
                                        T& s0, T& s1, T& s2) {
    s0 = s1 = s2 = (T)0;
    (void)n;
    if (v.src_on && i == v.src_i && j == v.src_j && k == v.src_k) {
        const T sv = (T)gld(&v.ctl->src_val);
        s0 = v.src_comp == 0 ? sv : (T)0;
        s1 = v.src_comp == 1 ? sv : (T)0;
        s2 = v.src_comp == 2 ? sv : (T)0;
    }
}

// Everything the E pass reads for one plane of a row: the Bloch state of the
// three sites, E^n, H^{n+1/2} and the H neighbours at y-1 and x-1.
template <typename T>
struct EPlane {
    BlochIn<T> b0, b1, b2;
    T ex, ey, ez, hx, hy, hz, hzy, hzx, hyx, hxy;
};

// The dense part of a plane (E and H of the cell, H at y-1 and x-1).
// Neighbours at y-1 only for j >= 1 and at x-1 only for i >= 1 (the offsets
// would wrap below zero otherwise).
template <typename T>
__device__ __forceinline__ void load_dense(EPlane<T>& p, const Fields<T>& f, uint32_t x, uint32_t sx, int i, int j) {
    p.hx = ldo(f.hn[0], x); p.hy = ldo(f.hn[1], x); p.hz = ldo(f.hn[2], x);
    p.hzy = j >= 1 ? ldo(f.hn[2], x - sx) : (T)0;
    p.hxy = j >= 1 ? ldo(f.hn[0], x - sx) : (T)0;
    p.hzx = i >= 1 ? ldo(f.hn[2], x - 1u) : (T)0;
    p.hyx = i >= 1 ? ldo(f.hn[1], x - 1u) : (T)0;
    p.ex = ldo(f.e[0], x); p.ey = ldo(f.e[1], x); p.ez = ldo(f.e[2], x);
}

// A whole plane: the Bloch state of its three sites and the dense part.
template <typename T>
__device__ __forceinline__ void load_plane(EPlane<T>& p, const Fields<T>& f, uint32_t x, uint32_t sx,
                                           uint32_t gi, bool g, bool inx, bool iny, bool inz, int i, int j) {
    p.b0 = bloch_load(f, 0, gi, g && inx);
    p.b1 = bloch_load(f, 1, gi, g && iny);
    p.b2 = bloch_load(f, 2, gi, g && inz);
    load_dense(p, f, x, sx, i, j);
}

// SPLIT selects what goes out one plane ahead: the whole next plane (false),
// or only its dense part, the Bloch state being loaded at the start of its
// own plane (true).  The whole plane keeps 90 VGPRs (5 waves per SIMD) and
// hides the Bloch loads behind a plane of work, which pays on small grids
// that leave most of the chip idle; the split keeps 76 (6 waves) and streams
// faster where the work fills the chip (a 320^3 batch; there the first pass
// also writes H with streaming stores, NT).
template <typename T, int TY, bool SPLIT>
__device__ __forceinline__ void curl_e_body(const SimView<T>& v, const Geom& gm, int w) {
    __shared__ double sh[TY];
    // the member's 1/eps_r table in LDS: one gather per plane fewer on the
    // vector memory path
    __shared__ T s_ie[kMaxMat];
    for (int q = (int)(threadIdx.x + 64 * threadIdx.y); q < kMaxMat; q += 64 * TY) s_ie[q] = gld(v.lut_inv_eps + q);
    __syncthreads();
    int bx, by, bz;
    decode_item(gm, w, bx, by, bz);
    const int i = bx * 64 + threadIdx.x;
    const int j = by * TY + threadIdx.y;
    const int64_t n = gld(&v.ctl->step);
    const int par = (int)(n & 1);
    const Fields<T> f = bind_fields(v, par);
    T* const tslot = tap_slot(v, n);
    double lsum = 0.0;
    const int kz0 = bz * gm.zseg, kz1 = min(kz0 + gm.zseg, v.nz);
    if (i < v.nx && j < v.ny) {
        const uint32_t sx = (uint32_t)v.sx, sxy = (uint32_t)v.sxy;
        uint32_t x = (uint32_t)i + sx * (uint32_t)j + sxy * (uint32_t)kz0;
        const bool iny0 = i >= 1, inz0 = i >= 1 && j >= 1;
        uint8_t m = ldo(v.mat, x);
        uint32_t gi = gain_index(v, bx, j, kz0, m >= kGainId, true);
        uint8_t m_n = (kz0 + 1 < kz1) ? ldo(v.mat, x + sxy) : (uint8_t)0;
        T hxm = kz0 >= 1 ? ldo(f.hn[0], x - sxy) : (T)0;
        T hym = kz0 >= 1 ? ldo(f.hn[1], x - sxy) : (T)0;
        // the x and y parts of the three sites' layer-table entries stay
        // fixed along the march in z (lay_coef_e: x at the half position for
        // Ex, y at the half position for Ey; the row j is wave-uniform)
        uint32_t txy0 = 0u, txy1 = 0u, txy2 = 0u;
        if (v.has_layer) {
            const uint32_t tx0 = lay_part(v, 0, 0, i), tx1 = lay_part(v, 0, 1, i);
            const int jw = __builtin_amdgcn_readfirstlane(j);
            const uint32_t ty0 = lay_part(v, 1, 0, jw), ty1 = lay_part(v, 1, 1, jw);
            txy0 = tx1 + ty0;
            txy1 = tx0 + ty1;
            txy2 = tx0 + ty0;
        }
        const LayC<T> h0 = lay_coef(v.lc, txy0), h1 = lay_coef(v.lc, txy1), h2 = lay_coef(v.lc, txy2);
        EPlane<T> P, Q;
        if constexpr (SPLIT) load_dense(P, f, x, sx, i, j);
        else load_plane(P, f, x, sx, gi, m >= kGainId, j >= 1 && kz0 >= 1, iny0 && kz0 >= 1, inz0, i, j);
        for (int k = kz0; k < kz1; ++k, x += sxy) {
            // software pipelining: the next plane's loads (its compact index
            // from the material byte read one plane earlier) go out before this
            // plane's arithmetic and stores, so two planes are in flight per
            // wave; with SPLIT the plane's own Bloch state goes out first.  The
            // wave issues them at raised priority, so that a wave about to
            // issue loads goes ahead of the others' arithmetic (0.3% on the
            // batch of 320^3 grids; the same in the H pass costs 0.9%)
            __builtin_amdgcn_s_setprio(2);
            if constexpr (SPLIT) {
                P.b0 = bloch_load(f, 0, gi, m >= kGainId && j >= 1 && k >= 1);
                P.b1 = bloch_load(f, 1, gi, m >= kGainId && iny0 && k >= 1);
                P.b2 = bloch_load(f, 2, gi, m >= kGainId && inz0);
            }
            uint32_t gi_n = 0;
            uint8_t m_nn = 0;
            if (k + 1 < kz1) {
                gi_n = gain_index(v, bx, j, k + 1, m_n >= kGainId, true);
                if (k + 2 < kz1) m_nn = ldo(v.mat, x + 2u * sxy);
                if constexpr (SPLIT) load_dense(Q, f, x + sxy, sx, i, j);
                else load_plane(Q, f, x + sxy, sx, gi_n, m_n >= kGainId, j >= 1, iny0, inz0, i, j);
            }
            __builtin_amdgcn_s_setprio(0);
            const bool g = m >= kGainId;
            const bool inx = (j >= 1 && k >= 1), iny = (i >= 1 && k >= 1), inz = (i >= 1 && j >= 1);
            const T ie = s_ie[m];
            T xi[3] = {(T)0, (T)0, (T)0};
            if (g && v.noise && (inx || iny || inz)) {
                const uint32_t cell = (uint32_t)(i + v.nx * (j + v.ny * k));
                noise3(v, cell, (uint32_t)n, xi);
            }
            T s0, s1, s2;
            source3(v, i, j, k, n, s0, s1, s2);
            // the z parts of this plane (0 without a layer and between the z
            // layers, where the column's coefficients taken before the march
            // apply)
            uint32_t tz0 = 0u, tz1 = 0u;
            if (v.has_layer && (k < v.lay_kz[0] || k >= v.lay_kz[1])) {
                tz0 = lay_part(v, 2, 0, k);
                tz1 = lay_part(v, 2, 1, k);
            }
            LayC<T> l0 = h0, l1 = h1, l2 = h2;
            if (tz0 | tz1) {
                l0 = lay_coef(v.lc, txy0 + tz0);
                l1 = lay_coef(v.lc, txy1 + tz0);
                l2 = lay_coef(v.lc, txy2 + tz1);
            }
            T acc = (T)0;
            {
                const T curl = inx ? dcurl(P.hz, P.hzy, P.hy, hym) : (T)0;
                const T en = bloch_site(v, f, 0, gi, P.ex, curl, ie, inx, g && inx, P.b0, xi[0], s0,
                                        l0, tslot);
                sto(f.en[0], x, en);
                if (tslot) sto(tslot, x, en);
                if (inx) acc += en * en;
            }
            {
                const T curl = iny ? dcurl(P.hx, hxm, P.hz, P.hzx) : (T)0;
                const T en = bloch_site(v, f, 1, gi, P.ey, curl, ie, iny, g && iny, P.b1, xi[1], s1,
                                        l1, tslot);
                sto(f.en[1], x, en);
                if (tslot) sto(tslot + v.tap_e, x, en);
                if (iny) acc += en * en;
            }
            {
                const T curl = inz ? dcurl(P.hy, P.hyx, P.hx, P.hxy) : (T)0;
                const T en = bloch_site(v, f, 2, gi, P.ez, curl, ie, inz, g && inz, P.b2, xi[2], s2,
                                        l2, tslot);
                sto(f.en[2], x, en);
                if (tslot) sto(tslot + 2 * v.tap_e, x, en);
                if (inz) acc += en * en;
            }
            if (v.box_on && i >= v.box[0] && i < v.box[3] && j >= v.box[1] && j < v.box[4] &&
                k >= v.box[2] && k < v.box[5])
                lsum += (double)acc;
            hxm = P.hx;
            hym = P.hy;
            P = Q;
            m = m_n;
            m_n = m_nn;
            gi = gi_n;
        }
    }
    if (v.box_on) {
        const double s = block_sum(lsum, sh);
        if (threadIdx.x == 0 && threadIdx.y == 0) sto(v.l_part, (uint32_t)w, s);
    }
}

// The tables are separate no-alias read-only arguments, so the compiler may
// keep the member's view in scalar registers across the kernel's stores.
template <typename T, int TY, bool SPLIT>
__global__ void __launch_bounds__(64 * TY) k_curl_e_batch(const SimView<T>* __restrict__ views,
                                                const Geom* __restrict__ geoms,
                                                const uint32_t* __restrict__ items, int nitems, int remap) {
    int r, w;
    batch_item(items, nitems, remap, r, w);
    curl_e_body<T, TY, SPLIT>(views[r], geoms[r], w);
}

// ------------------------------------------------ fused step (a1 to a5)
// Each wave owns one row (64 sites along x) of a 64 x TY tile and marches
// along z over a segment [z0, z1) of planes; after one barrier (the material
// tables into LDS) the waves never wait for each other and exchange no field
// values.  Per plane k a wave forms H^{n+1/2}(k) on its own
// row and stores it, forms again the two components of row j-1 that its E
// update needs (Hx, Hz), takes Hy and Hz at x-1 from the next lower lane (lane
// 0 forms them again at the tile edge), and then updates E, P and the
// populations of its row.  H^{n+1/2}(k-1) of its own row stays in registers;
// a segment that does not start at z = 0 first forms Hx, Hy of plane z0-1.
// Every recomputed value is the same expression on the same inputs as where
// it is owned (k_curl_h), so all kernel variants give bitwise identical fields.
template <typename T, int TY>
__device__ __forceinline__ void step_fused_body(const SimView<T>& v, const Geom& gm, int w) {
    __shared__ double sh[TY];
    // the member's eps_r and 1/eps_r tables in LDS: two gathers per plane
    // fewer on the vector memory path
    __shared__ T s_ie[kMaxMat], s_eps[kMaxMat];
    for (int q = (int)(threadIdx.x + 64 * threadIdx.y); q < kMaxMat; q += 64 * TY) {
        s_ie[q] = gld(v.lut_inv_eps + q);
        s_eps[q] = gld(v.lut_eps + q);
    }
    __syncthreads();
    int bx, by, bz;
    decode_item(gm, w, bx, by, bz);
    const int i = bx * 64 + threadIdx.x;
    const int j = by * TY + threadIdx.y;
    const int64_t n = gld(&v.ctl->step);
    const Fields<T> f = bind_fields(v, (int)(n & 1));
    T* const tslot = tap_slot(v, n);
    T wsum = (T)0;
    double lsum = 0.0;
    const int kz0 = bz * gm.zseg, kz1 = min(kz0 + gm.zseg, v.nz);
    if (j < v.ny) {                                   // wave-uniform
        const bool act = i < v.nx;
        const int ic = act ? i : v.nx;                // lanes past the grid read a valid site
        const uint32_t sx = (uint32_t)v.sx, sxy = (uint32_t)v.sxy;
        const T* __restrict__ Ex = f.e[0];
        const T* __restrict__ Ey = f.e[1];
        const T* __restrict__ Ez = f.e[2];
        const T* __restrict__ Hx0 = f.h[0];
        const T* __restrict__ Hy0 = f.h[1];
        const T* __restrict__ Hz0 = f.h[2];
        const bool up = j >= 1;                       // row j-1 exists (wave-uniform)
        const bool edge = threadIdx.x == 0 && i >= 1; // lane 0 of a tile past x = 0
        uint32_t x = (uint32_t)ic + sx * (uint32_t)j + sxy * (uint32_t)kz0;
        uint8_t m_next = ldo(v.mat, x);
        uint32_t gi_next = gain_index(v, bx, j, kz0, act && m_next >= kGainId, true);
        T ex = ldo(Ex, x), ey = ldo(Ey, x);           // E^n(k) of the row, carried along z
        T eym = up ? ldo(Ey, x - sx) : (T)0;          // Ey^n(k) of row j-1, carried along z
        // H^{n+1/2}(k-1) of the row: formed again at a segment start
        T hxp = (T)0, hyp = (T)0;
        if (kz0 >= 1) {
            const uint32_t xp = x - sxy;
            const T ezp = ldo(Ez, xp), eyp = ldo(Ey, xp), exp_ = ldo(Ex, xp);
            const T cx = dcurl(ldo(Ez, xp + sx), ezp, ey, eyp);
            const T cy = dcurl(ex, exp_, ldo(Ez, xp + 1u), ezp);
            hxp = h_update(ldo(Hx0, xp), v.S, cx, lay_coef_h(v, 0, ic, j, kz0 - 1));
            hyp = h_update(ldo(Hy0, xp), v.S, cy, lay_coef_h(v, 1, ic, j, kz0 - 1));
        }
        for (int k = kz0; k < kz1; ++k, x += sxy) {
            const uint8_t m = m_next;
            const uint32_t gi = gi_next;
            if (k + 1 < kz1) m_next = ldo(v.mat, x + sxy);     // one plane ahead
            const bool g = act && m >= kGainId;
            const bool inx = (j >= 1 && k >= 1), iny = (i >= 1 && k >= 1), inz = (i >= 1 && j >= 1);
            const BlochIn<T> b0 = bloch_load(f, 0, gi, g && inx);
            const BlochIn<T> b1 = bloch_load(f, 1, gi, g && iny);
            const BlochIn<T> b2 = bloch_load(f, 2, gi, g && inz);
            // ---- a1 on the own row
            const T ez = ldo(Ez, x);
            const T exk = ldo(Ex, x + sxy), eyk = ldo(Ey, x + sxy);
            const T hx = ldo(Hx0, x), hy = ldo(Hy0, x), hz = ldo(Hz0, x);
            const T cx = dcurl(ldo(Ez, x + sx), ez, eyk, ey);
            const T cy = dcurl(exk, ex, ldo(Ez, x + 1u), ez);
            const T cz = dcurl(ldo(Ey, x + 1u), ey, ldo(Ex, x + sx), ex);
            const LayC<T> ax = lay_coef_h(v, 0, ic, j, k);
            const LayC<T> ay = lay_coef_h(v, 1, ic, j, k);
            const LayC<T> az = lay_coef_h(v, 2, ic, j, k);
            const T nhx = h_update(hx, v.S, cx, ax);
            const T nhy = h_update(hy, v.S, cy, ay);
            const T nhz = h_update(hz, v.S, cz, az);
            if (act) {
                sto(f.hn[0], x, nhx);
                sto(f.hn[1], x, nhy);
                sto(f.hn[2], x, nhz);
                const T eps = s_eps[m];
                if (v.map != nullptr && k == v.map_k) plane_energy(v, i, j, eps, ex, ey, ez, nhx, nhy, nhz);
                T acc = (T)0;
                if (j >= 1 && k >= 1) acc += eps * ex * ex;
                if (i >= 1 && k >= 1) acc += eps * ey * ey;
                if (i >= 1 && j >= 1) acc += eps * ez * ez;
                if (i >= 1) acc += hx * nhx;
                if (j >= 1) acc += hy * nhy;
                if (k >= 1) acc += hz * nhz;
                wsum += (T)0.5 * acc;
            }
            // ---- Hx, Hz of row j-1 (its owner's expressions)
            T nhx_m = (T)0, nhz_m = (T)0, eymk = (T)0;
            if (up) {
                const uint32_t xm = x - sx;
                const T ezm = ldo(Ez, xm), exm = ldo(Ex, xm);
                eymk = ldo(Ey, xm + sxy);
                const T cxm = dcurl(ez, ezm, eymk, eym);
                const T czm = dcurl(ldo(Ey, xm + 1u), eym, ex, exm);
                nhx_m = h_update(ldo(Hx0, xm), v.S, cxm, lay_coef_h(v, 0, ic, j - 1, k));
                nhz_m = h_update(ldo(Hz0, xm), v.S, czm, lay_coef_h(v, 2, ic, j - 1, k));
            }
            // ---- Hy, Hz at x-1 of the own row
            T nhy_l = __shfl_up(nhy, 1, 64);
            T nhz_l = __shfl_up(nhz, 1, 64);
            if (edge) {
                const uint32_t xl = x - 1u;
                const T exl = ldo(Ex, xl), eyl = ldo(Ey, xl), ezl = ldo(Ez, xl);
                const T cyl = dcurl(ldo(Ex, xl + sxy), exl, ez, ezl);
                const T czl = dcurl(ey, eyl, ldo(Ex, xl + sx), exl);
                nhy_l = h_update(ldo(Hy0, xl), v.S, cyl, lay_coef_h(v, 1, i - 1, j, k));
                nhz_l = h_update(ldo(Hz0, xl), v.S, czl, lay_coef_h(v, 2, i - 1, j, k));
            }
            // ---- a2-a5 on the own row
            if (act) {
                const T ie = s_ie[m];
                T xi[3] = {(T)0, (T)0, (T)0};
                if (g && v.noise && (inx || iny || inz)) {
                    const uint32_t cell = (uint32_t)(i + v.nx * (j + v.ny * k));
                    noise3(v, cell, (uint32_t)n, xi);
                }
                T s0, s1, s2;
                source3(v, i, j, k, n, s0, s1, s2);
                T acc = (T)0;
                {
                    const T curl = inx ? dcurl(nhz, nhz_m, nhy, hyp) : (T)0;
                    const T en = bloch_site(v, f, 0, gi, ex, curl, ie, inx, g && inx, b0, xi[0], s0,
                                            lay_coef_e(v, 0, i, j, k), tslot);
                    sto(f.en[0], x, en);
                    if (tslot) sto(tslot, x, en);
                    if (inx) acc += en * en;
                }
                {
                    const T curl = iny ? dcurl(nhx, hxp, nhz, nhz_l) : (T)0;
                    const T en = bloch_site(v, f, 1, gi, ey, curl, ie, iny, g && iny, b1, xi[1], s1,
                                            lay_coef_e(v, 1, i, j, k), tslot);
                    sto(f.en[1], x, en);
                    if (tslot) sto(tslot + v.tap_e, x, en);
                    if (iny) acc += en * en;
                }
                {
                    const T curl = inz ? dcurl(nhy, nhy_l, nhx, nhx_m) : (T)0;
                    const T en = bloch_site(v, f, 2, gi, ez, curl, ie, inz, g && inz, b2, xi[2], s2,
                                            lay_coef_e(v, 2, i, j, k), tslot);
                    sto(f.en[2], x, en);
                    if (tslot) sto(tslot + 2 * v.tap_e, x, en);
                    if (inz) acc += en * en;
                }
                if (v.box_on && i >= v.box[0] && i < v.box[3] && j >= v.box[1] && j < v.box[4] &&
                    k >= v.box[2] && k < v.box[5])
                    lsum += (double)acc;
            }
            hxp = nhx;
            hyp = nhy;
            ex = exk;
            ey = eyk;
            eym = eymk;
            if (k + 1 < kz1) gi_next = gain_index(v, bx, j, k + 1, act && m_next >= kGainId, true);
        }
    }
    const double ws = block_sum((double)wsum, sh);
    __syncthreads();
    const double ls = v.box_on ? block_sum(lsum, sh) : 0.0;
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        sto(v.e_part, (uint32_t)w, ws);
        if (v.box_on) sto(v.l_part, (uint32_t)w, ls);
    }
}

// The tables are separate no-alias read-only arguments, so the compiler may
// keep the member's view in scalar registers across the kernel's stores.
template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY) k_step_fused_batch(const SimView<T>* __restrict__ views,
                                                const Geom* __restrict__ geoms,
                                                const uint32_t* __restrict__ items, int nitems, int remap) {
    int r, w;
    batch_item(items, nitems, remap, r, w);
    step_fused_body<T, TY>(views[r], geoms[r], w);
}


// Persistent form of the fused step: a grid sized to what the device holds at
// once drains the launch's work table from eight queues (queue x serves the
// entries x, x + 8, x + 16, ... that the dispatch order meant for XCD x, and
// workgroup b serves queue b mod 8, the XCD the hardware deals it to), so the
// XCD-aware order of the table survives.  Work items are independent within
// a step, so any order gives the same fields.  The queue counters are bumped
// by one lane with device-scope atomics; the last workgroup to leave zeroes
// all nine counters (eight queues and the leave count) for the next launch.
// Every workgroup leaves once its queue is empty, so the grid always drains.
template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY) k_step_fused_persist(const SimView<T>* __restrict__ views,
                                                              const Geom* __restrict__ geoms,
                                                              const uint32_t* __restrict__ items, int nitems,
                                                              uint32_t* __restrict__ queue) {
    __shared__ int s_pos;
    const bool lead = threadIdx.x == 0 && threadIdx.y == 0;
    const int qx = (int)(blockIdx.x & 7u);
    for (;;) {
        __syncthreads();                  // every wave is done with the previous item
        if (lead) s_pos = qx + 8 * (int)atomicAdd(queue + qx, 1u);
        __syncthreads();
        const int p = s_pos;
        if (p >= nitems) break;
        const uint32_t e = items[p];
        const int r = (int)(e >> 24), w = (int)(e & 0xFFFFFFu);
        step_fused_body<T, TY>(views[r], geoms[r], w);
    }
    if (lead && atomicAdd(queue + 8, 1u) == gridDim.x - 1u) {
        for (int q = 0; q < 9; ++q) atomicExch(queue + q, 0u);
    }
}

// ------------------------------------- fused step with LDS row exchange
// One pass over the fields per step (rows a1 to a5): H^{n+1/2} is formed,
// stored and handed to the E update of the same plane without being read back
// from memory.  A workgroup owns a tile of 64 x TY columns (one wave per row)
// and marches its waves together through a z segment, one barrier per plane:
//   before the barrier every wave forms H^{n+1/2}(k) of its row (its E^n(k+1)
//   loaded, E^n(k) carried from the previous plane, the +x and +y neighbours
//   read directly), stores it and puts Hx, Hz in LDS (double-buffered by the
//   plane's parity, so one barrier per plane suffices);
//   after it every wave updates E, P and the populations of its row at plane
//   k, taking Hx, Hz of row j-1 from LDS, Hy, Hz at x-1 from the next lower
//   lane and H^{n+1/2}(k-1) of its own row from registers.
// Values owned by another workgroup are formed again with their owner's
// expression: wave 0 forms Hx, Hz of row j0-1, lane 0 of every wave Hy, Hz of
// column i0-1, and a segment that does not start at z = 0 first forms Hx, Hy
// of plane z0-1; so every variant gives bitwise identical fields.
template <typename T, int TY>
__device__ __forceinline__ void step_lds_body(const SimView<T>& v, const Geom& gm, int w) {
    __shared__ double sh[TY];
    __shared__ T s_ie[kMaxMat], s_eps[kMaxMat];
    __shared__ T s_hx[2][TY][64], s_hz[2][TY][64];
    for (int q = (int)(threadIdx.x + 64 * threadIdx.y); q < kMaxMat; q += 64 * TY) {
        s_ie[q] = gld(v.lut_inv_eps + q);
        s_eps[q] = gld(v.lut_eps + q);
    }
    __syncthreads();
    int bx, by, bz;
    decode_item(gm, w, bx, by, bz);
    const int lane = (int)threadIdx.x, ty = (int)threadIdx.y;
    const int i = bx * 64 + lane;
    const int j = by * TY + ty;
    const int64_t n = gld(&v.ctl->step);
    const Fields<T> f = bind_fields(v, (int)(n & 1));
    T* const tslot = tap_slot(v, n);
    T wsum = (T)0;
    double lsum = 0.0;
    const int kz0 = bz * gm.zseg, kz1 = min(kz0 + gm.zseg, v.nz);
    const bool row = j < v.ny;                        // wave-uniform
    const bool act = row && i < v.nx;
    const int ic = i < v.nx ? i : v.nx;               // lanes past the grid read a valid site
    const uint32_t sx = (uint32_t)v.sx, sxy = (uint32_t)v.sxy;
    const T* __restrict__ Ex = f.e[0];
    const T* __restrict__ Ey = f.e[1];
    const T* __restrict__ Ez = f.e[2];
    const T* __restrict__ Hx0 = f.h[0];
    const T* __restrict__ Hy0 = f.h[1];
    const T* __restrict__ Hz0 = f.h[2];
    const bool halo_row = ty == 0 && j >= 1;          // wave 0 forms row j0-1 (wave-uniform)
    const bool halo_col = lane == 0 && i >= 1;        // lane 0 forms column i0-1
    uint32_t x = (uint32_t)ic + sx * (uint32_t)(row ? j : 0) + sxy * (uint32_t)kz0;
    uint8_t m_next = 0;
    uint32_t gi_next = 0;
    T ex = (T)0, ey = (T)0, ez = (T)0;                // E^n(k) of the row, carried along z
    T eym = (T)0;                                     // Ey^n(k) of row j0-1 (wave 0)
    T exl = (T)0;                                     // Ex^n(k) of column i0-1 (lane 0)
    T hxp = (T)0, hyp = (T)0;                         // H^{n+1/2}(k-1) of the row
    if (row) {
        m_next = ldo(v.mat, x);
        gi_next = gain_index(v, bx, j, kz0, act && m_next >= kGainId, true);
        ex = ldo(Ex, x);
        ey = ldo(Ey, x);
        ez = ldo(Ez, x);
        if (halo_row) eym = ldo(Ey, x - sx);
        if (halo_col) exl = ldo(Ex, x - 1u);
        if (kz0 >= 1) {                               // H^{n+1/2}(z0-1) of the row, formed again
            const uint32_t xp = x - sxy;
            const T ezp = ldo(Ez, xp), eyp = ldo(Ey, xp), exp_ = ldo(Ex, xp);
            const T cx = dcurl(ldo(Ez, xp + sx), ezp, ey, eyp);
            const T cy = dcurl(ex, exp_, ldo(Ez, xp + 1u), ezp);
            hxp = h_update(ldo(Hx0, xp), v.S, cx, lay_coef_h(v, 0, ic, j, kz0 - 1));
            hyp = h_update(ldo(Hy0, xp), v.S, cy, lay_coef_h(v, 1, ic, j, kz0 - 1));
        }
    }
    for (int k = kz0; k < kz1; ++k, x += sxy) {
        const int buf = k & 1;
        uint8_t m = 0;
        uint32_t gi = 0;
        T nhx = (T)0, nhy = (T)0, nhz = (T)0;         // H^{n+1/2}(k) of the row
        T nhx_m = (T)0, nhz_m = (T)0;                 // Hx, Hz of row j0-1 (wave 0)
        T nhy_l = (T)0, nhz_l = (T)0;                 // Hy, Hz of column i0-1 (lane 0)
        T exk = (T)0, eyk = (T)0, ezk = (T)0;         // E^n(k+1) of the row
        T eymk = (T)0, exlk = (T)0;
        BlochIn<T> b0{}, b1{}, b2{};
        bool g = false;
        const bool inx = (j >= 1 && k >= 1), iny = (i >= 1 && k >= 1), inz = (i >= 1 && j >= 1);
        if (row) {
            m = m_next;
            gi = gi_next;
            if (k + 1 < kz1) m_next = ldo(v.mat, x + sxy);
            g = act && m >= kGainId;
            b0 = bloch_load(f, 0, gi, g && inx);
            b1 = bloch_load(f, 1, gi, g && iny);
            b2 = bloch_load(f, 2, gi, g && inz);
            // ---- a1 on the own row (the H pass's expressions)
            exk = ldo(Ex, x + sxy);
            eyk = ldo(Ey, x + sxy);
            ezk = ldo(Ez, x + sxy);
            const T hx = ldo(Hx0, x), hy = ldo(Hy0, x), hz = ldo(Hz0, x);
            const T cx = dcurl(ldo(Ez, x + sx), ez, eyk, ey);
            const T cy = dcurl(exk, ex, ldo(Ez, x + 1u), ez);
            const T cz = dcurl(ldo(Ey, x + 1u), ey, ldo(Ex, x + sx), ex);
            nhx = h_update(hx, v.S, cx, lay_coef_h(v, 0, ic, j, k));
            nhy = h_update(hy, v.S, cy, lay_coef_h(v, 1, ic, j, k));
            nhz = h_update(hz, v.S, cz, lay_coef_h(v, 2, ic, j, k));
            s_hx[buf][ty][lane] = nhx;
            s_hz[buf][ty][lane] = nhz;
            if (act) {
                sto_nt(f.hn[0], x, nhx);
                sto_nt(f.hn[1], x, nhy);
                sto_nt(f.hn[2], x, nhz);
                const T eps = s_eps[m];
                if (v.map != nullptr && k == v.map_k) plane_energy(v, i, j, eps, ex, ey, ez, nhx, nhy, nhz);
                T acc = (T)0;
                if (j >= 1 && k >= 1) acc += eps * ex * ex;
                if (i >= 1 && k >= 1) acc += eps * ey * ey;
                if (i >= 1 && j >= 1) acc += eps * ez * ez;
                if (i >= 1) acc += hx * nhx;
                if (j >= 1) acc += hy * nhy;
                if (k >= 1) acc += hz * nhz;
                wsum += (T)0.5 * acc;
            }
            // ---- Hx, Hz of row j0-1 (its owner's expressions)
            if (halo_row) {
                const uint32_t xm = x - sx;
                const T ezm = ldo(Ez, xm), exm = ldo(Ex, xm);
                eymk = ldo(Ey, xm + sxy);
                const T cxm = dcurl(ez, ezm, eymk, eym);
                const T czm = dcurl(ldo(Ey, xm + 1u), eym, ex, exm);
                nhx_m = h_update(ldo(Hx0, xm), v.S, cxm, lay_coef_h(v, 0, ic, j - 1, k));
                nhz_m = h_update(ldo(Hz0, xm), v.S, czm, lay_coef_h(v, 2, ic, j - 1, k));
            }
            // ---- Hy, Hz of column i0-1
            if (halo_col) {
                const uint32_t xl = x - 1u;
                const T ezl = ldo(Ez, xl), eyl = ldo(Ey, xl);
                exlk = ldo(Ex, xl + sxy);
                const T cyl = dcurl(exlk, exl, ez, ezl);
                const T czl = dcurl(ey, eyl, ldo(Ex, xl + sx), exl);
                nhy_l = h_update(ldo(Hy0, xl), v.S, cyl, lay_coef_h(v, 1, i - 1, j, k));
                nhz_l = h_update(ldo(Hz0, xl), v.S, czl, lay_coef_h(v, 2, i - 1, j, k));
            }
        }
        __syncthreads();
        // ---- a2-a5 on the own row
        if (row) {
            const T hx_jm = ty >= 1 ? s_hx[buf][ty >= 1 ? ty - 1 : 0][lane] : nhx_m;
            const T hz_jm = ty >= 1 ? s_hz[buf][ty >= 1 ? ty - 1 : 0][lane] : nhz_m;
            T hy_im = __shfl_up(nhy, 1, 64);
            T hz_im = __shfl_up(nhz, 1, 64);
            if (lane == 0) {
                hy_im = nhy_l;
                hz_im = nhz_l;
            }
            if (act) {
                const T ie = s_ie[m];
                T xi[3] = {(T)0, (T)0, (T)0};
                if (g && v.noise && (inx || iny || inz)) {
                    const uint32_t cell = (uint32_t)(i + v.nx * (j + v.ny * k));
                    noise3(v, cell, (uint32_t)n, xi);
                }
                T s0, s1, s2;
                source3(v, i, j, k, n, s0, s1, s2);
                T acc = (T)0;
                {
                    const T curl = inx ? dcurl(nhz, hz_jm, nhy, hyp) : (T)0;
                    const T en = bloch_site(v, f, 0, gi, ex, curl, ie, inx, g && inx, b0, xi[0], s0,
                                            lay_coef_e(v, 0, i, j, k), tslot);
                    sto(f.en[0], x, en);
                    if (tslot) sto(tslot, x, en);
                    if (inx) acc += en * en;
                }
                {
                    const T curl = iny ? dcurl(nhx, hxp, nhz, hz_im) : (T)0;
                    const T en = bloch_site(v, f, 1, gi, ey, curl, ie, iny, g && iny, b1, xi[1], s1,
                                            lay_coef_e(v, 1, i, j, k), tslot);
                    sto(f.en[1], x, en);
                    if (tslot) sto(tslot + v.tap_e, x, en);
                    if (iny) acc += en * en;
                }
                {
                    const T curl = inz ? dcurl(nhy, hy_im, nhx, hx_jm) : (T)0;
                    const T en = bloch_site(v, f, 2, gi, ez, curl, ie, inz, g && inz, b2, xi[2], s2,
                                            lay_coef_e(v, 2, i, j, k), tslot);
                    sto(f.en[2], x, en);
                    if (tslot) sto(tslot + 2 * v.tap_e, x, en);
                    if (inz) acc += en * en;
                }
                if (v.box_on && i >= v.box[0] && i < v.box[3] && j >= v.box[1] && j < v.box[4] &&
                    k >= v.box[2] && k < v.box[5])
                    lsum += (double)acc;
            }
            hxp = nhx;
            hyp = nhy;
            ex = exk;
            ey = eyk;
            ez = ezk;
            eym = eymk;
            exl = exlk;
            if (k + 1 < kz1) gi_next = gain_index(v, bx, j, k + 1, act && m_next >= kGainId, true);
        }
    }
    const double ws = block_sum((double)wsum, sh);
    __syncthreads();
    const double ls = v.box_on ? block_sum(lsum, sh) : 0.0;
    if (threadIdx.x == 0 && threadIdx.y == 0) {
        sto(v.e_part, (uint32_t)w, ws);
        if (v.box_on) sto(v.l_part, (uint32_t)w, ls);
    }
}

template <typename T, int TY>
__global__ void __launch_bounds__(64 * TY) k_step_lds_batch(const SimView<T>* __restrict__ views,
                                                          const Geom* __restrict__ geoms,
                                                          const uint32_t* __restrict__ items, int nitems,
                                                          int remap) {
    int r, w;
    batch_item(items, nitems, remap, r, w);
    step_lds_body<T, TY>(views[r], geoms[r], w);
}

// ---------------------------------------------------------------- row a6
// First-order Mur on the wall E-sites of Mur axes.  Task (a, side, c) covers
// the sites of component c on the wall i_a = 0 or n_a.  A site that also lies
// on the wall of the third axis t belongs to the face applied last in x, y, z
// order; when that is face a (t < a) the neighbour it reads is itself a
// face-t site, whose new value is formed inline.  Sites on PEC walls stay 0.
__device__ __forceinline__ int sel3(int a, int x0, int x1, int x2) {
    return a == 0 ? x0 : (a == 1 ? x1 : x2);
}
__device__ __forceinline__ int64_t sel3(int a, int64_t x0, int64_t x1, int64_t x2) {
    return a == 0 ? x0 : (a == 1 ? x1 : x2);
}

template <typename T>
__device__ __forceinline__ void mur_body(const SimView<T>& v, int task) {
    if (task >= v.n_mur) return;
    const int code = (int)((v.mur_code >> (5 * task)) & 31u);
    const int a = code & 3, side = (code >> 2) & 1, c = (code >> 3) & 3;
    const int t = 3 - a - c;
    const int na = sel3(a, v.nx, v.ny, v.nz), nc = sel3(c, v.nx, v.ny, v.nz);
    const int ntd = sel3(t, v.nx, v.ny, v.nz);
    const int nt = ntd + 1;
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= (int64_t)nc * nt) return;
    const int u = (int)(q % nc);
    const int w = (int)(q / nc);
    const bool on_t = (w == 0 || w == ntd);
    const bool t_is_mur = ((v.mur_axes >> t) & 1) != 0;
    if (on_t && (!t_is_mur || t > a)) return;
    const int par = (int)(gld(&v.ctl->step) & 1);   // parity of the step being finished
    const Fields<T> f = bind_fields(v, par);
    const T* __restrict__ Ec = c == 0 ? f.e[0] : (c == 1 ? f.e[1] : f.e[2]);
    T* __restrict__ En = c == 0 ? f.en[0] : (c == 1 ? f.en[1] : f.en[2]);
    const int64_t sta = sel3(a, (int64_t)1, v.sx, v.sxy);
    const int64_t stc = sel3(c, (int64_t)1, v.sx, v.sxy);
    const int64_t stt = sel3(t, (int64_t)1, v.sx, v.sxy);
    const int wall = side ? na : 0;
    const int inner = side ? na - 1 : 1;
    const int64_t s = (int64_t)wall * sta + (int64_t)u * stc + (int64_t)w * stt;
    const int64_t s1 = s + (int64_t)(inner - wall) * sta;
    T e1new;
    if (!on_t) {
        e1new = En[s1];
    } else {
        const int tin = (w == 0) ? 1 : ntd - 1;
        const int64_t s2 = s1 + (int64_t)(tin - w) * stt;
        const T m1 = v.lut_mur[v.mat[s1]];
        e1new = Ec[s2] + m1 * (En[s2] - Ec[s1]);
    }
    const T m = v.lut_mur[v.mat[s]];
    En[s] = Ec[s1] + m * (e1new - Ec[s]);
}

template <typename T>
__global__ void __launch_bounds__(256) k_mur(SimView<T> v) {
    mur_body(v, (int)blockIdx.y);
}

// Batched: blockIdx.z is the member (members without Mur walls return).
template <typename T>
__global__ void __launch_bounds__(256) k_mur_batch(const SimView<T>* __restrict__ views) {
    mur_body(views[blockIdx.z], (int)blockIdx.y);
}

// ------------------------------------------------------ row a7, step end
// Sum of the per-workgroup partials in a fixed order: each thread keeps eight
// independent accumulators over a fixed stride (so its loads are in flight
// together), then a fixed tree over the threads; every thread gets the sum.
constexpr int kEndThreads = 1024;

__device__ __forceinline__ double sum_partials(const double* __restrict__ p, int n, double* sh) {
    const int t = threadIdx.x;
    double a[8] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    // accumulator r adds p[t + r K], p[t + (r + 8) K], ... in that order (K
    // threads); 32 loads go out per round.  Past the end they read as +0,
    // which changes no sum: an accumulator starts at +0 and so is never -0.
    for (int q = t; q < n; q += 32 * kEndThreads) {
        double v[32];
#pragma unroll
        for (int s = 0; s < 32; ++s) {
            const int e = q + s * kEndThreads;
            v[s] = e < n ? p[e] : 0.0;
        }
#pragma unroll
        for (int s = 0; s < 32; ++s) a[s & 7] += v[s];
    }
    double x = ((a[0] + a[1]) + (a[2] + a[3])) + ((a[4] + a[5]) + (a[6] + a[7]));
    x = wave_sum(x);
    if ((t & 63) == 0) sh[t >> 6] = x;
    __syncthreads();
    double r = 0.0;
    for (int w = 0; w < kEndThreads / 64; ++w) r += sh[w];
    return r;
}

template <typename T>
__device__ __forceinline__ void end_step_body(const SimView<T>& v) {
    __shared__ double sh[kEndThreads / 64];
    const int t = threadIdx.x;
    const int64_t n = gld(&v.ctl->step);
    const double W = sum_partials(v.e_part, v.n_part, sh);
    __syncthreads();
    const double L = v.box_on ? sum_partials(v.l_part, v.n_part, sh) : 0.0;
    const Fields<T> f = bind_fields(v, (int)(n & 1));
    for (int p = t; p < v.n_probes; p += kEndThreads) {
        const int c = v.probe_comp[p];
        const T* e = c == 0 ? f.en[0] : (c == 1 ? f.en[1] : f.en[2]);
        v.ring[(int64_t)p * v.decim + (n % v.decim)] = e[v.probe_off[p]];
    }
    if (t == 0) {
        if (!(W == W) || W - W != 0.0) v.ctl->nonfinite = 1;
        if (n < v.hist_cap) v.hist[n] = W;
        v.ctl->W_now = W;
        v.ctl->W_int += W;
        v.ctl->loss += L;
        v.ctl->step = n + 1;
        v.ctl->src_val = v.src_on ? (double)source_value(v, n + 1) : 0.0;
    }
}

template <typename T>
__global__ void __launch_bounds__(kEndThreads) k_end_step(SimView<T> v) {
    end_step_body(v);
}

// Batched: one workgroup per member.
template <typename T>
__global__ void __launch_bounds__(kEndThreads) k_end_step_batch(const SimView<T>* __restrict__ views) {
    end_step_body(views[blockIdx.x]);
}

// Source value of the current step (after the pump, a checkpoint load or a
// change of source), so that every step reads it from the control block.
template <typename T>
__global__ void k_source_init(SimView<T> v) {
    if (threadIdx.x == 0 && blockIdx.x == 0)
        v.ctl->src_val = v.src_on ? (double)source_value(v, v.ctl->step) : 0.0;
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
// Populations of the pump's initial state on interior gain E-sites (zero on
// the other components of a gain cell).  Grid (nbx, ny, nz) of one wave each.
template <typename T>
__global__ void __launch_bounds__(64) k_init_pop(SimView<T> v, T n1, T n2, T n3) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    const bool act = i < v.nx;
    const uint32_t x = (uint32_t)i + (uint32_t)v.sx * j + (uint32_t)v.sxy * k;
    const bool g = act && v.mat[act ? x : 0u] >= kGainId;
    const uint32_t gi = gain_index(v, (int)blockIdx.x, j, k, g, true);
    if (!g) return;
    const bool in[3] = {j >= 1 && k >= 1, i >= 1 && k >= 1, i >= 1 && j >= 1};
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        v.N[0][c][gi] = in[c] ? n1 : (T)0;
        v.N[1][c][gi] = in[c] ? n2 : (T)0;
        v.N[2][c][gi] = in[c] ? n3 : (T)0;
    }
}

// Record the current state (step n = ctl->step) into trajectory slot
// n - ctl->tap_base: E^n, P^n - P^{n-1} and N1 - N2, as the E pass does for
// the states it produces.  Grid (nbx, ny, nz) of one wave each.
template <typename T>
__global__ void __launch_bounds__(64) k_tap_state(SimView<T> v) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    const bool act = i < v.nx;
    const uint32_t x = (uint32_t)(act ? i : 0) + (uint32_t)v.sx * j + (uint32_t)v.sxy * k;
    const bool g = act && v.mat[x] >= kGainId;
    const uint32_t gi = gain_index(v, (int)blockIdx.x, j, k, g, true);
    if (!act) return;
    const int64_t n = gld(&v.ctl->step);
    const Fields<T> f = bind_fields(v, (int)(n & 1));
    T* slot = v.tap + (n - gld(&v.ctl->tap_base)) * v.tap_stride;
#pragma unroll
    for (int c = 0; c < 3; ++c) {
        sto(slot + c * v.tap_e, x, ldo(f.e[c], x));
        if (g) {
            sto(slot + 3 * v.tap_e + c * v.tap_c, gi, ldo(f.p[c], gi) - ldo(f.q[c], gi));
            sto(slot + 3 * v.tap_e + 3 * v.tap_c + c * v.tap_c, gi, ldo(f.n1[c], gi) - ldo(f.n2[c], gi));
        }
    }
}

// Dense copy of one compact Bloch-state array in the packed exchange layout
// (rows of nx+1 values, zero off the gain cells and on the upper walls, which
// the caller clears first), and the reverse.  Grid (nbx, ny, nz).
template <typename T>
__global__ void __launch_bounds__(64) k_gather(SimView<T> v, const T* __restrict__ src, T* __restrict__ dst) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    const bool act = i < v.nx;
    const uint32_t x = (uint32_t)i + (uint32_t)v.sx * j + (uint32_t)v.sxy * k;
    const bool g = act && v.mat[act ? x : 0u] >= kGainId;
    const uint32_t gi = gain_index(v, (int)blockIdx.x, j, k, g, true);
    if (act)
        dst[(int64_t)i + (int64_t)(v.nx + 1) * (j + (int64_t)(v.ny + 1) * k)] = g ? src[gi] : (T)0;
}

template <typename T>
__global__ void __launch_bounds__(64) k_scatter(SimView<T> v, const T* __restrict__ src, T* __restrict__ dst) {
    const int i = blockIdx.x * 64 + threadIdx.x, j = blockIdx.y, k = blockIdx.z;
    const bool act = i < v.nx;
    const uint32_t x = (uint32_t)i + (uint32_t)v.sx * j + (uint32_t)v.sxy * k;
    const bool g = act && v.mat[act ? x : 0u] >= kGainId;
    const uint32_t gi = gain_index(v, (int)blockIdx.x, j, k, g, true);
    if (g) dst[gi] = src[(int64_t)i + (int64_t)(v.nx + 1) * (j + (int64_t)(v.ny + 1) * k)];
}

}  // namespace mbf
