// exact.hip -- the exact reference forces of the accuracy measure (Eq. 20, Section 6.1.1).
//
// The error of a cutoff method is measured against the force of the full Lennard-Jones
// potential (Eq. 4) summed over every particle and every periodic image, which converges
// absolutely (the pair force falls as r^-7). Here the sum runs over all images within a
// radius R that may exceed half the box, so its only error is the part of the lattice sum
// beyond R (of order rho R^-4 on a particle at a planar interface). This is not on the
// per-step path: one lane per particle walks every box whose nearest point lies within R,
// image shift included, in the cell-sorted storage.
#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

inline unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

// floor division and remainder of an unwrapped box index
__device__ __forceinline__ void unwrap(int32_t u, int32_t N, int32_t &w, int32_t &img)
{
    img = u >= 0 ? u / N : -((-u + N - 1) / N);
    w = u - img * N;
}

__device__ __forceinline__ double gap(int32_t o, double h)
{
    // distance from a point of box 0 to box o along one axis is at least (|o| - 1) h
    const int32_t a = o < 0 ? -o : o;
    return a > 1 ? (double)(a - 1) * h : 0.0;
}

struct KForcesImages {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        PSet s;
        const uint32_t *cell_start;
        int64_t n;
        double R;
        double eps4;
        double eps24;
        double sig2;
        int32_t mx;
        int32_t my;
        int32_t mz;
        double *f_out;
        double *e_out;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KForcesImages::run(const Args &args_, uint32_t blk, uint32_t)
{
    Grid g = args_.g;
    PSet s = args_.s;
    const uint32_t *cell_start = args_.cell_start;
    int64_t n = args_.n;
    double R = args_.R;
    double eps4 = args_.eps4;
    double eps24 = args_.eps24;
    double sig2 = args_.sig2;
    int32_t mx = args_.mx;
    int32_t my = args_.my;
    int32_t mz = args_.mz;
    double *f_out = args_.f_out;
    double *e_out = args_.e_out;
    const int64_t p = (int64_t)blk * blockDim.x + threadIdx.x;
    if (p >= n) return;
    const double4 q = s.pos[p];
    const int32_t a = box_index(q.x, g.h[0], g.n[0]);
    const int32_t b = box_index(q.y, g.h[1], g.n[1]);
    const int32_t c = box_index(q.z, g.h[2], g.n[2]);
    const double R2 = R * R;
    double fx = 0.0, fy = 0.0, fz = 0.0, e = 0.0;
    for (int32_t oz = -mz; oz <= mz; ++oz) {
        const double gz = gap(oz, g.h[2]);
        if (gz * gz >= R2) continue;
        int32_t wc, iz;
        unwrap(c + oz, g.n[2], wc, iz);
        for (int32_t oy = -my; oy <= my; ++oy) {
            const double gy = gap(oy, g.h[1]);
            if (gz * gz + gy * gy >= R2) continue;
            int32_t wb, iy;
            unwrap(b + oy, g.n[1], wb, iy);
            for (int32_t ox = -mx; ox <= mx; ++ox) {
                const double gx = gap(ox, g.h[0]);
                if (gz * gz + gy * gy + gx * gx >= R2) continue;
                int32_t wa, ix;
                unwrap(a + ox, g.n[0], wa, ix);
                const double sx = (double)ix * g.L[0], sy = (double)iy * g.L[1], sz = (double)iz * g.L[2];
                const bool home = ix == 0 && iy == 0 && iz == 0;
                for (int32_t cq = 0; cq < (1 << g.sx); ++cq) {
                    const uint32_t key = cell_key(g, (wa << g.sx) + cq, wb, wc);
                    const uint32_t j0 = cell_start[key], j1 = cell_start[key + 1];
                    for (uint32_t j = j0; j < j1; ++j) {
                        if (home && (int64_t)j == p) continue;
                        const double4 o = s.pos[j];
                        const double dx = q.x - (o.x + sx), dy = q.y - (o.y + sy), dz = q.z - (o.z + sz);
                        const double r2 = dx * dx + dy * dy + dz * dz;
                        if (!(r2 < R2)) continue;
                        const double ir2 = 1.0 / r2;
                        const double s2 = sig2 * ir2;
                        const double s6 = s2 * s2 * s2;
                        const double s12 = s6 * s6;
                        const double fr = eps24 * (2.0 * s12 - s6) * ir2;
                        fx += fr * dx;
                        fy += fr * dy;
                        fz += fr * dz;
                        e += eps4 * (s12 - s6);
                    }
                }
            }
        }
    }
    const uint32_t id = s.id[p];
    if (f_out) {
        f_out[id] = fx;
        f_out[n + id] = fy;
        f_out[2 * n + id] = fz;
    }
    if (e_out) e_out[id] = 0.5 * e;
}

}  // namespace

int image_reach(double R, double h) { return (int)std::ceil(R / h) + 1; }

double image_box_visits(const Grid &g, int64_t n, double R)
{
    // boxes of the (2 m + 1)^3 offset cube per particle, an upper bound of the loop trips
    double v = (double)n;
    for (int k = 0; k < 3; ++k) v *= 2.0 * image_reach(R, g.h[k]) + 1.0;
    return v;
}

void launch_forces_images(const Grid &g, PSet s, const uint32_t *cell_start, int64_t n, double R,
                          double epsilon, double sigma, double *f_out, double *e_out, hipStream_t st)
{
    emit<KForcesImages>({g, s, cell_start, n, R, 4.0 * epsilon, 24.0 * epsilon, sigma * sigma,
                   image_reach(R, g.h[0]), image_reach(R, g.h[1]), image_reach(R, g.h[2]), f_out, e_out},
                   grid1(n), st);
}

}  // namespace dcm
