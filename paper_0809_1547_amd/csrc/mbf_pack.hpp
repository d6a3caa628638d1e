// Soft-sphere compression packing of the sample (Simulations section: the
// active medium fills the voids of a granular packing of spheres obtained by
// molecular dynamics).  Read as a compression run of soft spheres in a closed
// box in the dissipative (overdamped) limit of granular dynamics:
//
//   at scale s the spheres have diameters s d_i and the energy is
//     U_s = 1/2 sum_{i<j} (s (d_i + d_j)/2 - |x_i - x_j|)_+^2
//         + 1/2 sum_i sum_a [(s d_i/2 - x_ia)_+^2 + (x_ia + s d_i/2 - L_a)_+^2];
//   one step moves every centre along its force at once, x_i += eta F_i with
//   F_i = -grad_i U_s; s grows from s0 to 1 in `stages` equal steps with
//   `iters` steps at each scale below 1 and `final_iters` steps at s = 1.
//
// Only spheres closer than the largest diameter interact, so the box is cut
// into cells at least that wide and a sphere looks at the 27 cells around its
// own.  The centres sit in per-cell lists (one atomic slot each, at most
// kPackCap per cell), each sorted by sphere index.  A step gives each sphere 32
// lanes of a wave, one per neighbour cell: a lane adds the forces of its
// cell's spheres in list order, the lanes' sums are combined by a butterfly of
// fixed shape, and the first lane adds the walls, writes the new centre and
// bins it into the other cell table; a second launch sorts those lists (and
// clears the table the step read, for the step after).  Every run of the same
// input therefore gives the same bits.  Centres and diameters travel together
// as one 32-byte record (x, y, z, d), ping-ponged between two buffers.  FP64
// throughout.
#pragma once

#include "mbf_kernels.hpp"

namespace mbf {

constexpr int kPackCap = 32;        // centres one cell may hold
constexpr int kPackLanes = 32;      // lanes per sphere in the step (27 neighbour cells)
constexpr int kPackThreads = 256;   // 8 spheres per workgroup of the step
constexpr int kPackMaxCells = 1 << 24;

struct PackGrid {
    int g[3];          // cells per axis
    double w[3];       // cell widths, each at least the largest diameter
    double box[3];     // box edges L_a
    int ncell;
};

// Cell of one coordinate: floor(x / w) clamped to [0, g-1] (NaN -> 0).  The
// clamp keeps two centres closer than w at most one cell apart, so centres
// pushed slightly through a wall still find all their contacts.
__device__ __forceinline__ int pack_axis(double x, double w, int g) {
    const double q = x / w;
    if (!(q >= 1.0)) return 0;
    return (int)fmin(q, (double)(g - 1));
}

__device__ __forceinline__ int pack_cell(const PackGrid& gr, double4 p, int& cx, int& cy, int& cz) {
    cx = pack_axis(p.x, gr.w[0], gr.g[0]);
    cy = pack_axis(p.y, gr.w[1], gr.g[1]);
    cz = pack_axis(p.z, gr.w[2], gr.g[2]);
    return (cz * gr.g[1] + cy) * gr.g[0] + cx;
}

// Initial records from the caller's centres (n x 3) and diameters; both cell
// tables cleared.
__global__ void __launch_bounds__(256) k_pack_load(const double* __restrict__ x, const double* __restrict__ d, int n,
                                                   double4* __restrict__ P, int* __restrict__ cnt2, int ncell2) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    for (int c = i; c < ncell2; c += gridDim.x * 256) cnt2[c] = 0;
    if (i >= n) return;
    P[i] = make_double4(x[3 * i], x[3 * i + 1], x[3 * i + 2], d[i]);
}

__global__ void __launch_bounds__(64) k_pack_clear_flag(int* __restrict__ flag) {
    if (threadIdx.x == 0) flag[0] = 0;
}

__global__ void __launch_bounds__(256) k_pack_store(const double4* __restrict__ P, int n, double* __restrict__ x) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double4 p = P[i];
    x[3 * i] = p.x;
    x[3 * i + 1] = p.y;
    x[3 * i + 2] = p.z;
}

// One slot per sphere in its cell; a cell that would hold more than kPackCap
// centres raises *flag (sticky) and drops the extra ones.
__global__ void __launch_bounds__(256) k_pack_bin(const double4* __restrict__ P, int n, PackGrid gr,
                                                  int* __restrict__ cnt, int* __restrict__ lst, int* __restrict__ flag) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    int cx, cy, cz;
    const int c = pack_cell(gr, P[i], cx, cy, cz);
    const int slot = atomicAdd(cnt + c, 1);
    if (slot < kPackCap) lst[c * kPackCap + slot] = i;
    else atomicOr(flag, 1);
}

// Each cell's list in ascending sphere order (a sorting network in
// registers); also clears `clear` (ncell counts, the table the next step bins
// into).
__global__ void __launch_bounds__(256) k_pack_sort(const int* __restrict__ cnt, int* __restrict__ lst, int ncell,
                                                   int* __restrict__ clear) {
    const int c = blockIdx.x * 256 + threadIdx.x;
    if (c >= ncell) return;
    clear[c] = 0;
    const int k = min(cnt[c], kPackCap);
    if (k < 2) return;
    int* L = lst + c * kPackCap;
    int v[kPackCap];
#pragma unroll
    for (int t = 0; t < kPackCap; ++t) v[t] = t < k ? L[t] : 0x7fffffff;
    // odd-even transposition sort: kPackCap rounds of compare-exchange over
    // fixed register indices (no dynamic indexing, so nothing spills)
#pragma unroll
    for (int r = 0; r < kPackCap; ++r) {
#pragma unroll
        for (int t = r & 1; t + 1 < kPackCap; t += 2) {
            const int a = min(v[t], v[t + 1]), b = max(v[t], v[t + 1]);
            v[t] = a;
            v[t + 1] = b;
        }
    }
#pragma unroll
    for (int t = 0; t < kPackCap; ++t)
        if (t < k) L[t] = v[t];
}

// Pair force on sphere p from sphere q at scale s, added to f.
__device__ __forceinline__ void pack_pair(double4 p, double4 q, double s, double& fx, double& fy, double& fz) {
    const double rx = p.x - q.x, ry = p.y - q.y, rz = p.z - q.z;
    const double r2 = rx * rx + ry * ry + rz * rz;
    const double sig = s * (0.5 * (p.w + q.w));
    if (r2 > 0.0 && r2 < sig * sig) {
        const double r = sqrt(r2);
        const double k = (sig - r) / r;
        fx += k * rx;
        fy += k * ry;
        fz += k * rz;
    }
}

// Wall forces on one coordinate added to f: the x = 0 wall, then x = L.
__device__ __forceinline__ double pack_wall(double f, double x, double r, double L) {
    const double lo = r - x, hi = x + r - L;
    if (lo > 0.0) f += lo;
    if (hi > 0.0) f -= hi;
    return f;
}

// One step at scale s: Q_i = P_i + eta F_i, binned into (cnt_out, lst_out),
// whose counts start at zero.  Lane l < 27 of a sphere's 32 takes the
// neighbour cell (l / 9 - 1, l / 3 % 3 - 1, l % 3 - 1) in (z, y, x).
__global__ void __launch_bounds__(kPackThreads) k_pack_step(const double4* __restrict__ P, double4* __restrict__ Q,
                                                            int n, PackGrid gr, const int* __restrict__ cnt,
                                                            const int* __restrict__ lst, double s, double eta,
                                                            int* __restrict__ cnt_out, int* __restrict__ lst_out,
                                                            int* __restrict__ flag) {
    const int lane = (int)threadIdx.x & (kPackLanes - 1);
    const int i = (int)blockIdx.x * (kPackThreads / kPackLanes) + (int)threadIdx.x / kPackLanes;
    const bool act = i < n;
    double fx = 0.0, fy = 0.0, fz = 0.0;
    double4 p = make_double4(0.0, 0.0, 0.0, 0.0);
    if (act) {
        p = P[i];
        int cx, cy, cz;
        pack_cell(gr, p, cx, cy, cz);
        const int z = cz + lane / 9 - 1, y = cy + (lane / 3) % 3 - 1, x = cx + lane % 3 - 1;
        if (lane < 27 && z >= 0 && z < gr.g[2] && y >= 0 && y < gr.g[1] && x >= 0 && x < gr.g[0]) {
            const int c = (z * gr.g[1] + y) * gr.g[0] + x;
            const int k = min(cnt[c], kPackCap);
            const int* L = lst + c * kPackCap;
            for (int t = 0; t < k; ++t) {
                const int j = L[t];
                if (j != i) pack_pair(p, P[j], s, fx, fy, fz);
            }
        }
    }
    // butterfly over the sphere's 32 lanes: every lane ends with the same sum
#pragma unroll
    for (int o = kPackLanes / 2; o > 0; o >>= 1) {
        fx += __shfl_xor(fx, o, kPackLanes);
        fy += __shfl_xor(fy, o, kPackLanes);
        fz += __shfl_xor(fz, o, kPackLanes);
    }
    if (!act || lane != 0) return;
    const double r = s * (0.5 * p.w);
    fx = pack_wall(fx, p.x, r, gr.box[0]);
    fy = pack_wall(fy, p.y, r, gr.box[1]);
    fz = pack_wall(fz, p.z, r, gr.box[2]);
    const double4 q = make_double4(p.x + eta * fx, p.y + eta * fy, p.z + eta * fz, p.w);
    Q[i] = q;
    int cx, cy, cz;
    const int c = pack_cell(gr, q, cx, cy, cz);
    const int slot = atomicAdd(cnt_out + c, 1);
    if (slot < kPackCap) lst_out[c * kPackCap + slot] = i;
    else atomicOr(flag, 1);
}

// Per sphere: its share of U_1 (pairs with higher-indexed neighbours, its
// walls) and its largest overlap, into e[i], m[i].
__global__ void __launch_bounds__(256) k_pack_measure(const double4* __restrict__ P, int n, PackGrid gr,
                                                      const int* __restrict__ cnt, const int* __restrict__ lst,
                                                      double* __restrict__ e, double* __restrict__ m) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const double4 p = P[i];
    if (!(fabs(p.x) + fabs(p.y) + fabs(p.z) < INFINITY)) {   // a diverged run: NaN reaches the sum
        e[i] = NAN;
        m[i] = NAN;
        return;
    }
    int cx, cy, cz;
    pack_cell(gr, p, cx, cy, cz);
    double u = 0.0, mx = 0.0;
    for (int z = max(cz - 1, 0); z <= min(cz + 1, gr.g[2] - 1); ++z)
        for (int y = max(cy - 1, 0); y <= min(cy + 1, gr.g[1] - 1); ++y)
            for (int x = max(cx - 1, 0); x <= min(cx + 1, gr.g[0] - 1); ++x) {
                const int c = (z * gr.g[1] + y) * gr.g[0] + x;
                const int k = min(cnt[c], kPackCap);
                for (int t = 0; t < k; ++t) {
                    const int j = lst[c * kPackCap + t];
                    if (j <= i) continue;
                    const double4 q = P[j];
                    const double rx = p.x - q.x, ry = p.y - q.y, rz = p.z - q.z;
                    const double ov = 0.5 * (p.w + q.w) - sqrt(rx * rx + ry * ry + rz * rz);
                    if (ov > 0.0) {
                        u += 0.5 * ov * ov;
                        mx = fmax(mx, ov);
                    }
                }
            }
    const double r = 0.5 * p.w;
    const double xs[3] = {p.x, p.y, p.z};
#pragma unroll
    for (int a = 0; a < 3; ++a) {
        const double lo = r - xs[a], hi = xs[a] + r - gr.box[a];
        if (lo > 0.0) {
            u += 0.5 * lo * lo;
            mx = fmax(mx, lo);
        }
        if (hi > 0.0) {
            u += 0.5 * hi * hi;
            mx = fmax(mx, hi);
        }
    }
    e[i] = u;
    m[i] = mx;
}

// out[0] = sum e (each thread adds a strided share in order, then the shares
// are added in thread order), out[1] = max m; one workgroup of 256 threads.
__global__ void __launch_bounds__(256) k_pack_reduce(const double* __restrict__ e, const double* __restrict__ m, int n,
                                                     double* __restrict__ out) {
    __shared__ double su[256], sm[256];
    const int t = (int)threadIdx.x;
    double u = 0.0, mx = 0.0;
    for (int i = t; i < n; i += 256) {
        u += e[i];
        mx = fmax(mx, m[i]);
    }
    su[t] = u;
    sm[t] = mx;
    __syncthreads();
    if (t == 0) {
        double a = 0.0, b = 0.0;
        for (int k = 0; k < 256; ++k) {
            a += su[k];
            b = fmax(b, sm[k]);
        }
        out[0] = a;
        out[1] = b;
    }
}

}  // namespace mbf
