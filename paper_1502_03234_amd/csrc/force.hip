// force.hip -- Lennard-Jones force, energy and virial with per-particle cutoffs
// (Eq. 4; Section 3.2, Alg. 3.2: particle i uses the pair (i, j) iff |r_ij| < r_c[i] and only
// f_i is updated, so every ordered pair is visited from its own side -- a full list).
//
// One lane per particle, particles in cell-sorted order so that a wavefront holds a run of
// neighbouring boxes along x. Each candidate interval is scanned four slots at a time with all
// four loads issued before use (the loop is bound by memory latency otherwise; staging the
// rows through LDS measured slower). Lane i walks the box rows (fixed y, z) whose rectangle comes
// within r_c[i] of it; inside a row the candidate boxes are the x-interval that the sphere
// cuts, so the traversed volume follows the sphere at box resolution in y and z and exactly
// in x (the small-bin stencil idea of Fig. 13b taken to single boxes). Each candidate interval
// is a contiguous range of sorted slots. Periodic images are handled per interval: a wrapped
// interval adds the box edge to x_j, so dx = x_i - (x_j + shift) is the same number the
// minimum-image convention gives.
//
// 1/r^2 uses the hardware reciprocal refined by two Newton steps (error ~1 ulp). Energy and
// virial are accumulated per particle, reduced per workgroup in a fixed order, and the
// workgroup partials are summed in a fixed order by the reduction kernel.
#include "internal.h"

namespace dcm {

namespace {

constexpr int kForceBlock = 256;

__device__ __forceinline__ double rcp_refined(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ int floor_mul(double v, double inv_h) { return (int)floor(v * inv_h); }

// Conservative square root for box bounds: the hardware estimate, enlarged well past its error.
__device__ __forceinline__ double sqrt_up(double v) { return __builtin_amdgcn_sqrt(v) * (1.0 + 1e-6) + 1e-9; }

struct Acc {
    double fx, fy, fz, e, wxx, wyy, wzz, wxy, wxz, wyz, eshift;
    uint32_t pairs;
};

// Precision form: FP32 running sums with their TwoSum error terms (force, energy), plain FP32
// virial sums.
struct Acc32 {
    float fx, fy, fz, e, cfx, cfy, cfz, ce, wxx, wyy, wzz, wxy, wxz, wyz, eshift;
    uint32_t pairs;
};

// s + x with the rounding error of the addition collected in c (Knuth's TwoSum: exact for any
// magnitudes, no branch).
__device__ __forceinline__ void two_sum_add(float &s, float &c, float x)
{
    const float t = s + x;
    const float bp = t - s;
    const float ap = t - bp;
    c += (s - ap) + (x - bp);
    s = t;
}

__device__ __forceinline__ float rcp_f32(float a)
{
    float y = __builtin_amdgcn_rcpf(a);
    return fmaf(y, fmaf(-a, y, 1.0f), y);
}

template <int PAIR, bool SHIFT, bool IMAGE>
__device__ __forceinline__ void interact(const ForceArgs &a, const double4 pj, bool valid,
                                         double xi, double yi, double zi, double rci, double rc2,
                                         double sx, double sy, double sz, Acc &c)
{
    // x_j moved to the periodic image of its interval (adding 0 is exact, so the no-image
    // variant gives the same bits without the three additions)
    double dx = IMAGE ? xi - (pj.x + sx) : xi - pj.x;
    double dy = IMAGE ? yi - (pj.y + sy) : yi - pj.y;
    double dz = IMAGE ? zi - (pj.z + sz) : zi - pj.z;
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double lim2 = rc2;
    if (PAIR == DCM_PAIR_MAX) {
        double rcp = pj.w > rci ? pj.w : rci;
        lim2 = rcp * rcp;
    }
    if (valid && r2 < lim2) {
        double inv = rcp_refined(r2);
        double sr2 = a.sigma2 * inv;
        double sr6 = sr2 * sr2 * sr2;
        double fr = a.eps24 * sr6 * fma(2.0, sr6, -1.0) * inv;
        double fxp = fr * dx, fyp = fr * dy, fzp = fr * dz;
        c.fx += fxp;
        c.fy += fyp;
        c.fz += fzp;
        c.e += fma(sr6, sr6, -sr6);
        c.wxx = fma(dx, fxp, c.wxx);
        c.wyy = fma(dy, fyp, c.wyy);
        c.wzz = fma(dz, fzp, c.wzz);
        c.wxy = fma(dx, fyp, c.wxy);
        c.wxz = fma(dx, fzp, c.wxz);
        c.wyz = fma(dy, fzp, c.wyz);
        c.pairs += 1;
        if (SHIFT && PAIR == DCM_PAIR_MAX) {
            double s2 = a.sigma2 / lim2;
            double s6 = s2 * s2 * s2;
            c.eshift += fma(s6, s6, -s6);
        }
    }
}

template <int PAIR, bool SHIFT, bool IMAGE>
__device__ __forceinline__ void interact(const ForceArgs &a, const double4 pj, bool valid,
                                         double xi, double yi, double zi, double rci, double rc2,
                                         double sx, double sy, double sz, Acc32 &c)
{
    // displacement, r^2 and the cutoff test stay FP64: the pair set is the FP64 one
    double dx = IMAGE ? xi - (pj.x + sx) : xi - pj.x;
    double dy = IMAGE ? yi - (pj.y + sy) : yi - pj.y;
    double dz = IMAGE ? zi - (pj.z + sz) : zi - pj.z;
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double lim2 = rc2;
    if (PAIR == DCM_PAIR_MAX) {
        double rcp = pj.w > rci ? pj.w : rci;
        lim2 = rcp * rcp;
    }
    if (valid && r2 < lim2) {
        const float fdx = (float)dx, fdy = (float)dy, fdz = (float)dz;
        const float inv = rcp_f32((float)r2);
        const float sr2 = a.sigma2f * inv;
        const float sr6 = sr2 * sr2 * sr2;
        const float fr = a.eps24f * sr6 * fmaf(2.0f, sr6, -1.0f) * inv;
        const float fxp = fr * fdx, fyp = fr * fdy, fzp = fr * fdz;
        two_sum_add(c.fx, c.cfx, fxp);
        two_sum_add(c.fy, c.cfy, fyp);
        two_sum_add(c.fz, c.cfz, fzp);
        two_sum_add(c.e, c.ce, fmaf(sr6, sr6, -sr6));
        c.wxx = fmaf(fdx, fxp, c.wxx);
        c.wyy = fmaf(fdy, fyp, c.wyy);
        c.wzz = fmaf(fdz, fzp, c.wzz);
        c.wxy = fmaf(fdx, fyp, c.wxy);
        c.wxz = fmaf(fdx, fzp, c.wxz);
        c.wyz = fmaf(fdy, fzp, c.wyz);
        c.pairs += 1;
        if (SHIFT && PAIR == DCM_PAIR_MAX) {
            const float s2 = a.sigma2f / (float)lim2;
            const float s6 = s2 * s2 * s2;
            c.eshift += fmaf(s6, s6, -s6);
        }
    }
}

// All candidates of one slot interval [jb, je), U loads in flight at a time; the particle
// itself (slot i) is skipped.
template <int PAIR, bool SHIFT, bool IMAGE, int U, typename A>
__device__ __forceinline__ void scan(const ForceArgs &a, uint32_t jb, uint32_t je, int64_t i,
                                     double xi, double yi, double zi, double rci, double rc2,
                                     double sx, double sy, double sz, A &c)
{
    for (uint32_t j0 = jb; j0 < je; j0 += U) {
        const uint32_t last = je - 1;
        double4 p[U];
        uint32_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            jj[u] = j0 + u < je ? j0 + u : last;
            p[u] = a.pos[jj[u]];
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            interact<PAIR, SHIFT, IMAGE>(a, p[u], j0 + u < je && jj[u] != i, xi, yi, zi, rci, rc2, sx, sy, sz, c);
    }
}

template <int PAIR, bool SHIFT, int U, typename A>
__device__ __forceinline__ void scan_interval(const ForceArgs &a, uint32_t jb, uint32_t je, int64_t i,
                                              double xi, double yi, double zi, double rci, double rc2,
                                              double sx, double sy, double sz, A &c)
{
    const bool image = sx != 0.0 || sy != 0.0 || sz != 0.0;
    if (__any(image))
        scan<PAIR, SHIFT, true, U, A>(a, jb, je, i, xi, yi, zi, rci, rc2, sx, sy, sz, c);
    else
        scan<PAIR, SHIFT, false, U, A>(a, jb, je, i, xi, yi, zi, rci, rc2, sx, sy, sz, c);
}

// Walks the box rows within particle i's search radius and scans each row's x-interval.
template <int PAIR, bool SHIFT, int U, typename A>
__device__ __forceinline__ void traverse(const ForceArgs &a, int64_t i, double xi, double yi, double zi,
                                         double rci, double rc2, double rc_max, A &c)
{
    const Grid &g = a.grid;
    // search radius (slightly enlarged so that rounding in the box bounds never drops a box
    // that holds an in-range particle; the pair test itself is exact)
    double rs = PAIR == DCM_PAIR_MAX ? rc_max : rci;
    rs = rs * (1.0 + 1e-12) + 1e-9;
    const double rs2 = rs * rs;
    const double ihx = 1.0 / g.h[0], ihy = 1.0 / g.h[1], ihz = 1.0 / g.h[2];
    const int izlo = floor_mul(zi - rs, ihz), izhi = floor_mul(zi + rs, ihz);
    for (int iz = izlo; iz <= izhi; ++iz) {
        const double zlo = iz * g.h[2];
        const double dzm = fmax(0.0, fmax(zlo - zi, zi - (zlo + g.h[2])));
        const double remz = rs2 - dzm * dzm;
        if (remz < 0.0) continue;
        int wz = iz;
        double sz = 0.0;
        if (iz < 0) { wz += g.n[2]; sz = -g.L[2]; }
        else if (iz >= g.n[2]) { wz -= g.n[2]; sz = g.L[2]; }
        const double ry = sqrt_up(remz);
        const int iylo = floor_mul(yi - ry, ihy), iyhi = floor_mul(yi + ry, ihy);
        for (int iy = iylo; iy <= iyhi; ++iy) {
            const double ylo = iy * g.h[1];
            const double dym = fmax(0.0, fmax(ylo - yi, yi - (ylo + g.h[1])));
            const double rem = remz - dym * dym;
            if (rem < 0.0) continue;
            int wy = iy;
            double sy = 0.0;
            if (iy < 0) { wy += g.n[1]; sy = -g.L[1]; }
            else if (iy >= g.n[1]) { wy -= g.n[1]; sy = g.L[1]; }
            const double rx = sqrt_up(rem);
            const int ixlo = floor_mul(xi - rx, ihx), ixhi = floor_mul(xi + rx, ihx);
            const int64_t row = ((int64_t)wz * g.n[1] + wy) * g.n[0];
            // up to two contiguous slot ranges (the second one wraps around x)
            int lo0 = ixlo, hi0 = ixhi, lo1 = 0, hi1 = -1;
            double sx0 = 0.0, sx1 = 0.0;
            if (ixlo < 0) {
                lo0 = ixlo + g.n[0]; hi0 = g.n[0] - 1; sx0 = -g.L[0];
                lo1 = 0; hi1 = ixhi;
            } else if (ixhi >= g.n[0]) {
                hi0 = g.n[0] - 1;
                lo1 = 0; hi1 = ixhi - g.n[0]; sx1 = g.L[0];
            }
            scan_interval<PAIR, SHIFT, U, A>(a, a.cell_start[row + lo0], a.cell_start[row + hi0 + 1], i, xi, yi,
                                             zi, rci, rc2, sx0, sy, sz, c);
            if (hi1 >= lo1)
                scan_interval<PAIR, SHIFT, U, A>(a, a.cell_start[row + lo1], a.cell_start[row + hi1 + 1], i, xi,
                                                 yi, zi, rci, rc2, sx1, sy, sz, c);
        }
    }
}

template <int PAIR, bool SHIFT, int U, int PREC>
__global__ void __launch_bounds__(kForceBlock) k_forces(ForceArgs a, double rc_max)
{
    // hardware (round-robin over XCDs) block order: the cost per particle varies strongly
    // with z through the cutoffs, and interleaving keeps every XCD's share of it even
    const int64_t b = blockIdx.x;
    const int64_t i = b * kForceBlock + threadIdx.x;
    Acc c = {};
    if (i < a.n) {
        const double4 pi = a.pos[i];
        const double xi = pi.x, yi = pi.y, zi = pi.z, rci = pi.w;
        const double rc2 = rci * rci;
        // a non-finite position or a cutoff outside (0, rc_max] would send the box loops out
        // of the grid: such a particle gets no traversal and a NaN force (flagged below)
        const bool sane = isfinite(xi) && isfinite(yi) && isfinite(zi) && rci > 0.0 && rci <= rc_max;
        if (PREC == DCM_FP64) {
            if (sane) traverse<PAIR, SHIFT, U, Acc>(a, i, xi, yi, zi, rci, rc2, rc_max, c);
        } else {
            Acc32 c32 = {};
            if (sane) traverse<PAIR, SHIFT, U, Acc32>(a, i, xi, yi, zi, rci, rc2, rc_max, c32);
            // FP32 sums and their compensation terms, combined in FP64
            c.fx = (double)c32.fx + (double)c32.cfx;
            c.fy = (double)c32.fy + (double)c32.cfy;
            c.fz = (double)c32.fz + (double)c32.cfz;
            c.e = (double)c32.e + (double)c32.ce;
            c.wxx = c32.wxx; c.wyy = c32.wyy; c.wzz = c32.wzz;
            c.wxy = c32.wxy; c.wxz = c32.wxz; c.wyz = c32.wyz;
            c.eshift = c32.eshift;
            c.pairs = c32.pairs;
        }
        if (!sane) c.fx = NAN;
        // e_i = 1/2 sum 4 eps (sr12 - sr6); W_i = 1/2 sum dx (x) f
        double e = 0.5 * a.eps4 * c.e;
        if (SHIFT) {
            if (PAIR == DCM_PAIR_MAX) e -= 0.5 * a.eps4 * c.eshift;
            else {
                double s2 = a.sigma2 / rc2;
                double s6 = s2 * s2 * s2;
                e -= 0.5 * (double)c.pairs * (a.eps4 * (s6 * s6 - s6));
            }
        }
        c.e = e;
        c.wxx *= 0.5; c.wyy *= 0.5; c.wzz *= 0.5;
        c.wxy *= 0.5; c.wxz *= 0.5; c.wyz *= 0.5;
        a.fx[i] = c.fx;
        a.fy[i] = c.fy;
        a.fz[i] = c.fz;
        if (!(isfinite(c.fx) && isfinite(c.fy) && isfinite(c.fz))) atomicOr(a.flags, kFlagNonFinite);
        if (a.e_out || a.w_out || a.pairs_out) {
            const uint32_t id = a.id[i];
            if (a.e_out) a.e_out[id] = e;
            if (a.w_out) {
                a.w_out[0 * a.n + id] = c.wxx;
                a.w_out[1 * a.n + id] = c.wyy;
                a.w_out[2 * a.n + id] = c.wzz;
                a.w_out[3 * a.n + id] = c.wxy;
                a.w_out[4 * a.n + id] = c.wxz;
                a.w_out[5 * a.n + id] = c.wyz;
            }
            if (a.pairs_out) a.pairs_out[id] = c.pairs;
        }
    }
    // fixed-order workgroup reduction of e, W and the pair count
    double v[7] = {c.e, c.wxx, c.wyy, c.wzz, c.wxy, c.wxz, c.wyz};
    long long pc = c.pairs;
#pragma unroll
    for (int q = 0; q < 7; ++q)
        for (int off = 32; off > 0; off >>= 1) v[q] += __shfl_xor(v[q], off, 64);
    for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
    __shared__ double lds[kForceBlock / 64][8];
    __shared__ long long ldp[kForceBlock / 64];
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int q = 0; q < 7; ++q) lds[w][q] = v[q];
        ldp[w] = pc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial p = {};
        for (int q = 0; q < kForceBlock / 64; ++q) {
            p.e += lds[q][0];
            for (int r = 0; r < 6; ++r) p.w[r] += lds[q][1 + r];
            p.pairs += ldp[q];
        }
        a.partials[b] = p;
    }
}

}  // namespace

int force_blocks(int64_t n) { return (int)((n + kForceBlock - 1) / kForceBlock); }

template <int PREC>
static void launch_prec(const ForceArgs &a, int nb, hipStream_t st)
{
    constexpr int U = 4;
    const double rc_max = a.rc_max;
    if (a.pair_rule == DCM_PAIR_MAX) {
        if (a.energy_shift) hipLaunchKernelGGL((k_forces<DCM_PAIR_MAX, true, U, PREC>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
        else hipLaunchKernelGGL((k_forces<DCM_PAIR_MAX, false, U, PREC>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
    } else {
        if (a.energy_shift) hipLaunchKernelGGL((k_forces<DCM_PAIR_I, true, U, PREC>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
        else hipLaunchKernelGGL((k_forces<DCM_PAIR_I, false, U, PREC>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
    }
}

void launch_forces(const ForceArgs &a, hipStream_t st)
{
    const int nb = force_blocks(a.n);
    if (a.precision == DCM_FP32C) launch_prec<DCM_FP32C>(a, nb, st);
    else launch_prec<DCM_FP64>(a, nb, st);
}

}  // namespace dcm
