// mumford_shah.hip -- two-phase piecewise-constant Mumford-Shah segmentation (Eq. 13).
//
// Eq. 13 with its data terms in the intended pairing (liquid set against rho_l, vapor set
// against rho_v) and the densities fixed at the two-means centres (Eq. 14). The labelling
// is found through the convex relaxation over u in [0, 1] (u = 1 liquid):
//     sum_c u_c r_c + sum_c sum_k w_k |u(c + e_k) - u(c)|,  r_c = (f_c - 1)^2 - (f_c - rho_v / rho_l)^2,
// with f = image / rho_l and w_k = nu L_max / h_k (lengths in units of the longest box edge,
// energy per unit box volume). The perimeter term is the anisotropic total variation over the
// faces of the periodic box grid, for which the level set {u > 1/2} of a minimiser is a
// minimising labelling (coarea formula; Chan, Esedoglu and Nikolova 2006). The relaxation is
// solved by the primal-dual algorithm of Chambolle and Pock (2011, Algorithm 1, theta = 1),
// steps sigma = tau = 1 / sqrt(12), from the threshold labelling, for a fixed number of
// iterations:
//     dual     p_k <- clamp(p_k + sigma (ubar(c + e_k) - ubar(c)), -w_k, w_k)
//     primal   u'  <- clamp(u - tau (r - div p), 0, 1),  div p = sum_k p_k(c) - p_k(c - e_k)
//              ubar <- 2 u' - u,  u <- u'
// then liquid iff u > 1/2. Both updates are per-box stencils of the previous iterate, so the
// result does not depend on the order boxes are visited; with contraction into fused
// multiply-adds off, every box takes the operations of the plain loop in the same order and
// the labels are reproducible bit for bit.
//
// One thread per box, two launches per iteration; each reads its stencil from HBM (L2 keeps
// the neighbour planes), the dual 56 B and the primal 56 B per box.
#include "internal.h"
#include "launch.h"

#pragma clang fp contract(off)

namespace dcm {

namespace {

inline unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ void coords3(const Grid &g, int64_t c, int32_t &i, int32_t &j, int32_t &k)
{
    const uint32_t u = (uint32_t)c, nx = (uint32_t)g.n[0], ny = (uint32_t)g.n[1];
    const uint32_t r = u / nx;
    i = (int32_t)(u - r * nx);
    k = (int32_t)(r / ny);
    j = (int32_t)(r - (uint32_t)k * ny);
}

__device__ __forceinline__ int64_t at(const Grid &g, int32_t i, int32_t j, int32_t k)
{
    return ((int64_t)k * g.n[1] + j) * g.n[0] + i;
}

__device__ __forceinline__ double clamp(double v, double lo, double hi) { return fmin(fmax(v, lo), hi); }

// u, ubar from the threshold labels; p = 0; the data term r.
struct KMsInit {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        int64_t G;
        const uint32_t *img;
        const double *km;
        const uint8_t *raw;
        MsWork m;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t nblk);
};

__device__ void KMsInit::run(const Args &a, uint32_t blk, uint32_t)
{
    const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
    if (c >= a.G) return;
    const double rl = a.km[1];
    double r = 0.0;
    if (rl > 0.0) {
        const double cv = a.km[0] / rl;
        const double f = (double)a.img[c] / rl;
        const double fl = f - 1.0, fv = f - cv;
        r = fl * fl - fv * fv;
    }
    const double u = a.raw[c] == kLabelLiquid ? 1.0 : 0.0;
    a.m.r[c] = r;
    a.m.u[c] = u;
    a.m.ub[c] = u;
    a.m.p[c] = 0.0;
    a.m.p[a.G + c] = 0.0;
    a.m.p[2 * a.G + c] = 0.0;
}

struct KMsDual {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        MsWork m;
        double sigma;
        double w[3];
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t nblk);
};

__device__ void KMsDual::run(const Args &a, uint32_t blk, uint32_t)
{
    const Grid &g = a.g;
    const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
    if (c >= g.G) return;
    int32_t i, j, k;
    coords3(g, c, i, j, k);
    const int64_t nb[3] = {at(g, i + 1 == g.n[0] ? 0 : i + 1, j, k), at(g, i, j + 1 == g.n[1] ? 0 : j + 1, k),
                           at(g, i, j, k + 1 == g.n[2] ? 0 : k + 1)};
    const double u0 = a.m.ub[c];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
        const double v = a.m.p[q * g.G + c] + a.sigma * (a.m.ub[nb[q]] - u0);
        a.m.p[q * g.G + c] = clamp(v, -a.w[q], a.w[q]);
    }
}

struct KMsPrimal {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        MsWork m;
        double tau;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t nblk);
};

__device__ void KMsPrimal::run(const Args &a, uint32_t blk, uint32_t)
{
    const Grid &g = a.g;
    const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
    if (c >= g.G) return;
    int32_t i, j, k;
    coords3(g, c, i, j, k);
    const int64_t G = g.G;
    const int64_t bx = at(g, i == 0 ? g.n[0] - 1 : i - 1, j, k), by = at(g, i, j == 0 ? g.n[1] - 1 : j - 1, k),
                  bz = at(g, i, j, k == 0 ? g.n[2] - 1 : k - 1);
    const double *p = a.m.p;
    const double div = ((p[c] - p[bx]) + (p[G + c] - p[G + by])) + (p[2 * G + c] - p[2 * G + bz]);
    const double u = a.m.u[c];
    const double un = clamp(u - a.tau * (a.m.r[c] - div), 0.0, 1.0);
    a.m.ub[c] = 2.0 * un - u;
    a.m.u[c] = un;
}

struct KMsLabel {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        int64_t G;
        const double *km;
        const double *u;
        uint8_t *raw;
        uint8_t *label;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t nblk);
};

__device__ void KMsLabel::run(const Args &a, uint32_t blk, uint32_t)
{
    const int64_t c = (int64_t)blk * kBlock + threadIdx.x;
    if (c >= a.G) return;
    if (!(a.km[1] > 0.0)) return;            // empty image: the threshold labels stay
    const uint8_t s = a.u[c] > 0.5 ? kLabelLiquid : kLabelVapor;
    a.raw[c] = s;
    a.label[c] = s;
}

}  // namespace

void launch_mumford_shah(const Grid &g, const uint32_t *img, const double *km, const MsParams &ms, uint8_t *raw,
                         uint8_t *label, MsWork m, hipStream_t st)
{
    const double sigma = 1.0 / std::sqrt(12.0), tau = sigma;
    KMsDual::Args da;
    da.g = g;
    da.m = m;
    da.sigma = sigma;
    for (int q = 0; q < 3; ++q) da.w[q] = ms.nu * ms.Lmax / g.h[q];
    emit<KMsInit>({g.G, img, km, raw, m}, grid1(g.G), st);
    for (int32_t it = 0; it < ms.iters; ++it) {
        emit<KMsDual>(da, grid1(g.G), st);
        emit<KMsPrimal>({g, m, tau}, grid1(g.G), st);
    }
    emit<KMsLabel>({g.G, km, m.u, raw, label}, grid1(g.G), st);
}

}  // namespace dcm
