/*
 * FP64 CPU oracle of the soft-sphere packing of the sample.
 *
 * TEST INFRASTRUCTURE ONLY: loaded by the test-suite, never by the product
 * library, with which it shares no source.
 *
 * The sample is a granular packing of dielectric spheres obtained by
 * molecular dynamics (Simulations section; the packing method itself is
 * deferred to earlier work).  It is read here as a compression run of soft
 * spheres in a closed box, in the dissipative (overdamped) limit of granular
 * dynamics:
 *
 *   spheres i = 0..n-1, diameters d_i, centres x_i in the box [0, L]^3 (cell
 *   units); at scale s the diameters are s d_i and the energy is
 *     U_s(x) = 1/2 sum_{i<j} (s (d_i + d_j)/2 - |x_i - x_j|)_+^2
 *            + 1/2 sum_i sum_a [(s d_i/2 - x_ia)_+^2 + (x_ia + s d_i/2 - L_a)_+^2]
 *   one step moves every centre along its force at once:
 *     x_i <- x_i + eta F_i(x),   F_i = -grad_i U_s
 *   schedule: s_m = s0 + (1 - s0) m / stages for m = 0..stages; `iters` steps
 *   at each s_m with m < stages, then `final_iters` steps at s = 1.  With
 *   stages = 0 the run is `final_iters` steps at s = 1.
 *
 * F_i is the plain sum over every other sphere j in ascending order, then the
 * six walls.  Coincident centres exert no force on each other (the direction
 * is undefined).  OpenMP splits the spheres; each sphere's sum stays in order.
 */
#include <math.h>
#include <stdlib.h>

static void pack_force(int n, const double* box, const double* d, const double* x, double s, double* f) {
#pragma omp parallel for schedule(static)
    for (int i = 0; i < n; ++i) {
        double fx = 0.0, fy = 0.0, fz = 0.0;
        for (int j = 0; j < n; ++j) {
            if (j == i) continue;
            const double rx = x[3 * i] - x[3 * j];
            const double ry = x[3 * i + 1] - x[3 * j + 1];
            const double rz = x[3 * i + 2] - x[3 * j + 2];
            const double r2 = rx * rx + ry * ry + rz * rz;
            const double sig = s * (0.5 * (d[i] + d[j]));
            if (r2 > 0.0 && r2 < sig * sig) {
                const double r = sqrt(r2);
                const double q = (sig - r) / r;
                fx += q * rx;
                fy += q * ry;
                fz += q * rz;
            }
        }
        const double ri = s * (0.5 * d[i]);
        double fa[3] = {fx, fy, fz};
        for (int a = 0; a < 3; ++a) {
            const double lo = ri - x[3 * i + a];
            const double hi = x[3 * i + a] + ri - box[a];
            if (lo > 0.0) fa[a] += lo;
            if (hi > 0.0) fa[a] -= hi;
        }
        f[3 * i] = fa[0];
        f[3 * i + 1] = fa[1];
        f[3 * i + 2] = fa[2];
    }
}

/* Runs the schedule on x (n x 3, updated in place).  Returns 0, or -1 on bad
   arguments or when out of memory. */
int orc_pack_md(int n, const double* box, const double* d, double* x, double s0, int stages, int iters,
                int final_iters, double eta) {
    if (n < 0 || stages < 0 || iters < 0 || final_iters < 0) return -1;
    if (n == 0) return 0;
    double* f = (double*)malloc(sizeof(double) * 3 * (size_t)n);
    if (!f) return -1;
    for (int m = 0; m <= stages; ++m) {
        const double s = stages > 0 ? s0 + (1.0 - s0) * (double)m / (double)stages : 1.0;
        const int steps = m < stages ? iters : final_iters;
        for (int t = 0; t < steps; ++t) {
            pack_force(n, box, d, x, s, f);
            for (int k = 0; k < 3 * n; ++k) x[k] += eta * f[k];
        }
    }
    free(f);
    return 0;
}

/* U_s(x) and the largest overlap (of a pair, or of a sphere with a wall) at
   scale s: out[0] = U, out[1] = max overlap (0 when nothing overlaps). */
void orc_pack_energy(int n, const double* box, const double* d, const double* x, double s, double* out) {
    double u = 0.0, mx = 0.0;
    for (int i = 0; i < n; ++i) {
        for (int j = i + 1; j < n; ++j) {
            const double rx = x[3 * i] - x[3 * j];
            const double ry = x[3 * i + 1] - x[3 * j + 1];
            const double rz = x[3 * i + 2] - x[3 * j + 2];
            const double ov = s * (0.5 * (d[i] + d[j])) - sqrt(rx * rx + ry * ry + rz * rz);
            if (ov > 0.0) {
                u += 0.5 * ov * ov;
                if (ov > mx) mx = ov;
            }
        }
        const double ri = s * (0.5 * d[i]);
        for (int a = 0; a < 3; ++a) {
            const double lo = ri - x[3 * i + a];
            const double hi = x[3 * i + a] + ri - box[a];
            if (lo > 0.0) {
                u += 0.5 * lo * lo;
                if (lo > mx) mx = lo;
            }
            if (hi > 0.0) {
                u += 0.5 * hi * hi;
                if (hi > mx) mx = hi;
            }
        }
    }
    out[0] = u;
    out[1] = mx;
}
