// force.hip -- Lennard-Jones force, energy and virial with per-particle cutoffs
// (Eq. 4; Section 3.2, Alg. 3.2: particle i uses the pair (i, j) iff |r_ij| < r_c[i] and only
// f_i is updated, so every ordered pair is visited from its own side -- a full list).
//
// One lane per particle, particles in cell-sorted order so that a wavefront holds a run of
// neighbouring boxes along x. Lane i walks the box rows (fixed y, z) whose rectangle comes
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

// Workgroups are dealt round-robin to the 8 XCDs; give each XCD a contiguous range of
// logical blocks so that neighbouring particles share one L2.
__device__ __forceinline__ int64_t xcd_remap(int64_t p, int64_t nblk)
{
    constexpr int64_t kXcd = 8;
    int64_t q = nblk / kXcd, r = nblk % kXcd;
    int64_t xcd = p % kXcd, local = p / kXcd;
    return xcd < r ? xcd * (q + 1) + local : r * (q + 1) + (xcd - r) * q + local;
}

__device__ __forceinline__ double rcp_refined(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    y = fma(y, e, y);
    e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ int floor_div(double v, double h) { return (int)floor(v / h); }

struct Acc {
    double fx, fy, fz, e, wxx, wyy, wzz, wxy, wxz, wyz, eshift;
    uint32_t pairs;
};

template <int PAIR, bool SHIFT>
__device__ __forceinline__ void interact(const ForceArgs &a, const double4 pj, int64_t i, int64_t j,
                                         double xi, double yi, double zi, double rci, double rc2,
                                         double sx, double sy, double sz, Acc &c)
{
    double dx = xi - (pj.x + sx);
    double dy = yi - (pj.y + sy);
    double dz = zi - (pj.z + sz);
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    double lim2 = rc2;
    if (PAIR == DCM_PAIR_MAX) {
        double rcp = pj.w > rci ? pj.w : rci;
        lim2 = rcp * rcp;
    }
    if (r2 < lim2 && j != i) {
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

template <int PAIR, bool SHIFT>
__global__ void __launch_bounds__(kForceBlock) k_forces(ForceArgs a, double rc_max)
{
    const int64_t nblk = gridDim.x;
    const int64_t b = xcd_remap(blockIdx.x, nblk);
    const int64_t i = b * kForceBlock + threadIdx.x;
    const Grid &g = a.grid;
    Acc c = {};
    if (i < a.n) {
        const double4 pi = a.pos[i];
        const double xi = pi.x, yi = pi.y, zi = pi.z, rci = pi.w;
        const double rc2 = rci * rci;
        // a non-finite position or a cutoff outside (0, rc_max] would send the box loops out
        // of the grid: such a particle gets no traversal and a NaN force (flagged below)
        const bool sane = isfinite(xi) && isfinite(yi) && isfinite(zi) && rci > 0.0 && rci <= rc_max;
        if (!sane) c.fx = NAN;
        // search radius (slightly enlarged so that rounding in the box bounds never drops a
        // box that holds an in-range particle; the pair test itself is exact)
        double rs = PAIR == DCM_PAIR_MAX ? rc_max : rci;
        rs = rs * (1.0 + 1e-12) + 1e-9;
        const double rs2 = rs * rs;
        const int izlo = sane ? floor_div(zi - rs, g.h[2]) : 0;
        const int izhi = sane ? floor_div(zi + rs, g.h[2]) : -1;
        for (int iz = izlo; iz <= izhi; ++iz) {
            const double zlo = iz * g.h[2];
            const double dzm = fmax(0.0, fmax(zlo - zi, zi - (zlo + g.h[2])));
            const double remz = rs2 - dzm * dzm;
            if (remz < 0.0) continue;
            int wz = iz;
            double sz = 0.0;
            if (iz < 0) { wz += g.n[2]; sz = -g.L[2]; }
            else if (iz >= g.n[2]) { wz -= g.n[2]; sz = g.L[2]; }
            const double ry = sqrt(remz);
            const int iylo = floor_div(yi - ry, g.h[1]), iyhi = floor_div(yi + ry, g.h[1]);
            for (int iy = iylo; iy <= iyhi; ++iy) {
                const double ylo = iy * g.h[1];
                const double dym = fmax(0.0, fmax(ylo - yi, yi - (ylo + g.h[1])));
                const double rem = remz - dym * dym;
                if (rem < 0.0) continue;
                int wy = iy;
                double sy = 0.0;
                if (iy < 0) { wy += g.n[1]; sy = -g.L[1]; }
                else if (iy >= g.n[1]) { wy -= g.n[1]; sy = g.L[1]; }
                const double rx = sqrt(rem);
                const int ixlo = floor_div(xi - rx, g.h[0]), ixhi = floor_div(xi + rx, g.h[0]);
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
                {
                    const uint32_t jb = a.cell_start[row + lo0], je = a.cell_start[row + hi0 + 1];
                    for (uint32_t j = jb; j < je; ++j)
                        interact<PAIR, SHIFT>(a, a.pos[j], i, j, xi, yi, zi, rci, rc2, sx0, sy, sz, c);
                }
                if (hi1 >= lo1) {
                    const uint32_t jb = a.cell_start[row + lo1], je = a.cell_start[row + hi1 + 1];
                    for (uint32_t j = jb; j < je; ++j)
                        interact<PAIR, SHIFT>(a, a.pos[j], i, j, xi, yi, zi, rci, rc2, sx1, sy, sz, c);
                }
            }
        }
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

void launch_forces(const ForceArgs &a, hipStream_t st)
{
    const int nb = force_blocks(a.n);
    const double rc_max = a.rc_max;
    if (a.pair_rule == DCM_PAIR_MAX) {
        if (a.energy_shift) hipLaunchKernelGGL((k_forces<DCM_PAIR_MAX, true>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
        else hipLaunchKernelGGL((k_forces<DCM_PAIR_MAX, false>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
    } else {
        if (a.energy_shift) hipLaunchKernelGGL((k_forces<DCM_PAIR_I, true>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
        else hipLaunchKernelGGL((k_forces<DCM_PAIR_I, false>), dim3(nb), dim3(kForceBlock), 0, st, a, rc_max);
    }
}

}  // namespace dcm
