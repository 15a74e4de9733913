// tail.hip -- runtime tail correction of the dynamic cutoff (Section 7, Eq. 21-22).
//
// Eq. 22 gives particle i the pair energy its cutoff r_c[i] leaves out: the Lennard-Jones
// energy integrated over the points beyond r_c[i], weighted by the liquid density in the liquid
// and the vapor density in the vapor. The force added is the same integral of the pair force
// (Eq. 21 applied under the integral, over the pairs beyond the cutoff), so that the cutoff
// force plus the correction approaches the full force.
//
// The two phases around i are modelled by a plane at signed distance delta (> 0: i in the
// liquid), the liquid on the side of the unit normal m. With a = max(r_c, |delta|) and the
// radial integrals of the pair energy V
//     W(a)  = int_a^inf r V dr   = 4 eps sigma^2 [(sigma/a)^10 / 10 - (sigma/a)^4 / 4]
//     U2(a) = int_a^inf r^2 V dr = 4 eps sigma^3 [(sigma/a)^9 / 9  - (sigma/a)^3 / 3]
// the integrals over the liquid part of each shell (a cap of area 2 pi r (r + delta) and first
// moment pi (r^2 - delta^2) once r > |delta|) close to
//     F  = m (rho_l - rho_v) pi [-V(a) (a^2 - delta^2) - 2 W(a)]
//     du = rho_v 4 pi U2(r_c) + (rho_l - rho_v) L(delta),
//     L  = 4 pi [U2(r_c) - U2(a)] + 2 pi [U2(a) + delta W(a)]   (delta > 0)
//     L  = 2 pi [U2(a) + delta W(a)]                             (delta <= 0).
// delta and m come from the signed box field phi = (depth into the liquid) - h/2 on liquid
// boxes and -(depth into the vapor - h/2) on vapor boxes (h/2 the mean half box edge): the
// interface sits midway between the last liquid and the first vapor box centre. delta is the
// trilinear interpolant of phi at x_i (Eq. 6) and m the interpolant's gradient (a distance
// field has a unit gradient; where the field flattens at the band limit the force fades with
// it). If all eight boxes around x_i are at the band limit (the capped depth less a relative
// 1e-9, so that rounding in the distances cannot move the decision), i is deep in its phase:
// du is that phase's uniform value and F = 0. Densities are the two-means centres (Eq. 14)
// over the box volume, divided by 64 per smoothing pass (a pass multiplies a uniform image by 4
// along each axis).
//
// One lane per particle in storage order, after the pair-force kernel of the same force
// evaluation: the force is added to f_i, du_i / 2 to the particle's energy and, in a
// fixed-order block sum, to the force kernel's per-block energy partial (same blocks).
#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

constexpr int kTailBlock = 64;   // the pair-force kernel's block, so that partial b is shared

__device__ __forceinline__ double lerp(double a, double b, double t) { return a + t * (b - a); }

struct KTail {
    static constexpr int kThreads = kTailBlock, kWaves = 0;
    using Args = TailArgs;
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KTail::run(const Args &a, uint32_t blk, uint32_t)
{
    const Grid &g = a.grid;
    const int64_t i = (int64_t)blk * kTailBlock + threadIdx.x;
    double half_du = 0.0;
    if (i < a.n) {
        const double4 q = a.pos[i];
        const double x[3] = {q.x, q.y, q.z};
        const double rc = q.w;
        int64_t i0[3], i1[3];
        double t[3];
        for (int k = 0; k < 3; ++k) {
            double u = x[k] / g.h[k] - 0.5;
            if (!isfinite(u)) u = 0.0;                 // keeps the gathers inside the grid
            const double f = floor(u);
            t[k] = u - f;
            int64_t fi = (int64_t)f % g.n[k];
            if (fi < 0) fi += g.n[k];
            i0[k] = fi;
            i1[k] = fi + 1 == g.n[k] ? 0 : fi + 1;
        }
        const double cap = a.cap, s = a.half_edge, lim = (cap - s) * (1.0 - 1e-9);
        // phi[c][b][a]: corner (i_a, j_b, k_c)
        double phi[2][2][2];
        bool deep = true;
#pragma unroll
        for (int c = 0; c < 2; ++c)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int e = 0; e < 2; ++e) {
                    const int64_t box = ((c ? i1[2] : i0[2]) * g.n[1] + (b ? i1[1] : i0[1])) * g.n[0] +
                                        (e ? i1[0] : i0[0]);
                    const double dl = fmin(a.dist_l[box], cap);
                    const double v = dl > 0.0 ? dl - s : -(fmin(a.dist_v[box], cap) - s);
                    phi[c][b][e] = v;
                    deep = deep && fabs(v) >= lim;
                }
        const double rho_v = a.km[0] * a.inv_norm, rho_l = a.km[1] * a.inv_norm;
        const double e4 = 4.0 * a.epsilon, sg = a.sigma;
        const double pi = 3.14159265358979323846;
        // U2(rc) and the uniform tail 4 pi U2(rc)
        const double src = sg / rc, src3 = src * src * src, src9 = src3 * src3 * src3;
        const double u2rc = e4 * sg * sg * sg * (src9 / 9.0 - src3 / 3.0);
        const double whole = 4.0 * pi * u2rc;
        double du, fxi = 0.0, fyi = 0.0, fzi = 0.0;
        if (deep) {
            du = (phi[0][0][0] > 0.0 ? rho_l : rho_v) * whole;
        } else {
            const double c00 = lerp(phi[0][0][0], phi[0][0][1], t[0]);
            const double c10 = lerp(phi[0][1][0], phi[0][1][1], t[0]);
            const double c01 = lerp(phi[1][0][0], phi[1][0][1], t[0]);
            const double c11 = lerp(phi[1][1][0], phi[1][1][1], t[0]);
            const double delta = lerp(lerp(c00, c10, t[1]), lerp(c01, c11, t[1]), t[2]);
            // gradient of the trilinear interpolant
            const double gx = lerp(lerp(phi[0][0][1] - phi[0][0][0], phi[0][1][1] - phi[0][1][0], t[1]),
                                   lerp(phi[1][0][1] - phi[1][0][0], phi[1][1][1] - phi[1][1][0], t[1]), t[2]) / g.h[0];
            const double gy = lerp(lerp(phi[0][1][0] - phi[0][0][0], phi[0][1][1] - phi[0][0][1], t[0]),
                                   lerp(phi[1][1][0] - phi[1][0][0], phi[1][1][1] - phi[1][0][1], t[0]), t[2]) / g.h[1];
            const double gz = lerp(lerp(phi[1][0][0] - phi[0][0][0], phi[1][0][1] - phi[0][0][1], t[0]),
                                   lerp(phi[1][1][0] - phi[0][1][0], phi[1][1][1] - phi[0][1][1], t[0]), t[1]) / g.h[2];
            const double ad = fabs(delta), aa = fmax(rc, ad);
            const double sa = sg / aa, sa2 = sa * sa, sa3 = sa2 * sa, sa4 = sa2 * sa2, sa6 = sa3 * sa3;
            const double va = e4 * (sa6 * sa6 - sa6);
            const double wa = e4 * sg * sg * (sa6 * sa4 / 10.0 - sa4 / 4.0);
            const double u2a = e4 * sg * sg * sg * (sa6 * sa3 / 9.0 - sa3 / 3.0);
            const double drho = rho_l - rho_v;
            double liq = 2.0 * pi * (u2a + delta * wa);
            if (delta > 0.0) liq += 4.0 * pi * (u2rc - u2a);
            du = rho_v * whole + drho * liq;
            const double fn = drho * pi * (-va * (aa * aa - delta * delta) - 2.0 * wa);
            fxi = fn * gx;
            fyi = fn * gy;
            fzi = fn * gz;
        }
        a.fx[i] += fxi;
        a.fy[i] += fyi;
        a.fz[i] += fzi;
        half_du = 0.5 * du;
        if (a.e_out) a.e_out[a.id[i]] += half_du;
    }
    // fixed-order block sum into the force kernel's energy partial of this block
    double v = half_du;
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    __shared__ double lds[kTailBlock / 64];
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    if (threadIdx.x == 0) {
        double sum = 0.0;
        for (int w = 0; w < kTailBlock / 64; ++w) sum += lds[w];
        a.partials[blk].e += sum;
    }
}

}  // namespace

void launch_tail(const TailArgs &a, hipStream_t st)
{
    emit<KTail>(a, (uint32_t)((a.n + kTailBlock - 1) / kTailBlock), st);
}

}  // namespace dcm
