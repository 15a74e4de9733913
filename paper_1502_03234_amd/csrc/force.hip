// force.hip -- Lennard-Jones force, energy and virial with per-particle cutoffs
// (Eq. 4; Section 3.2, Alg. 3.2: particle i uses the pair (i, j) iff |r_ij| < r_c[i] and only
// f_i is updated, so every ordered pair is visited from its own side -- a full list).
//
// One lane per particle, particles in storage (sort-key) order, so a wavefront holds a run of
// neighbouring boxes along x inside one force row. A force row is a block of 2 x 2 boxes in y
// and z (1 x 1 where an axis is too short or odd; see cell_key), and storage order keeps the boxes
// of a force row and any x-interval in one contiguous slot range. Lane i walks the force rows
// whose y-z rectangle comes within r_c[i] of it and, in each, scans the slot range of the
// x-interval the sphere cuts: the small-bin stencil of Fig. 13b with single-box resolution in
// x. Grouping rows in y and z trades some extra candidates for a third of the row steps and far
// better L2 reuse between neighbouring waves. The row loops are uniform over the wave, in row
// offsets relative to each lane's own force row, so the lanes of one row scan the same
// neighbour rows together. Candidates are loaded four at a time with all loads issued before
// use (the loop is bound by memory latency otherwise), through a buffer descriptor of the
// position array: 32-bit offsets, and the up to three slots read past an interval's end need no
// clamp (reads beyond the array return zeros; such slots are masked out). Periodic images are handled per
// interval: a wrapped interval adds the box edge to x_j, so dx = x_i - (x_j + shift) is the same
// number the minimum-image convention gives.
//
// 1/r^2 uses the hardware reciprocal refined by one Newton step (the estimate carries about half
// the FP64 bits; one step squares its relative error, leaving a few ulp). Energy and virial are
// accumulated per particle, reduced per workgroup in a fixed order, and the workgroup partials
// are summed in a fixed order by the reduction kernel.
#include <climits>
#include <type_traits>

#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

// One wave per workgroup: waves differ widely in cost (their particles' cutoffs differ), and a
// wider workgroup would hold a finished wave's slot until its slowest sibling is done (256
// threads: 2.07 ms per launch on the 2M slab; 128: 1.98; 64: 1.95).
constexpr int kForceBlock = 64;

__device__ __forceinline__ double rcp_refined(double a)
{
    double y = __builtin_amdgcn_rcp(a);
    double e = fma(-a, y, 1.0);
    return fma(y, e, y);
}

__device__ __forceinline__ int floor_mul(double v, double inv_h) { return (int)floor(v * inv_h); }

// Conservative square root for box bounds: the hardware estimate, enlarged well past its error.
__device__ __forceinline__ double sqrt_up(double v) { return __builtin_amdgcn_sqrt(v) * (1.0 + 1e-6) + 1e-9; }

// An upper bound of sqrt_up(v) for every v <= rs * rs: the largest half-width of a row's x-interval
// for search radius rs.
__device__ __forceinline__ double x_reach(double rs) { return rs * (1.0 + 1e-5) + 1e-8; }

// FP64 form. The pair loop accumulates the force and the virial in units of 24 eps sigma^6 (the
// factor is applied once per particle) and, in place of the energy, the sum of r^-6: with
// s = (sigma/r)^6 the force scalar is 24 eps s (2 s - 1) / r^2, so the trace of the virial sum is
// sum (2 s^2 - s) / sigma^6 (up to rounding), and sum (s^2 - s) = sigma^6 (trace - sum r^-6) / 2
// gives the energy without a per-pair term of its own. For sigma = 1 every scaling is exact.
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
                                         double sx, double sy, double sz, Acc &c, uint32_t)
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
        // in units of sigma^6: u = r^-6, so (sigma / r)^6 = sigma^6 u and the force scalar
        // 24 eps (sigma / r)^6 (2 (sigma / r)^6 - 1) / r^2 is 24 eps sigma^6 times fr
        double inv = rcp_refined(r2);
        double u = inv * inv * inv;
        double fr = u * fma(a.sigma6x2, u, -1.0) * inv;
        double fxp = fr * dx, fyp = fr * dy, fzp = fr * dz;
        c.fx += fxp;
        c.fy += fyp;
        c.fz += fzp;
        c.e += u;
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
                                         double sx, double sy, double sz, Acc32 &c, uint32_t)
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

// List building: appends the slots within the list radius (rc2 holds its square) to
// list[count * n + i]; counts past the capacity are kept to flag the overflow.
struct AccList {
    uint32_t *list;
    int64_t n, i;
    uint32_t cap, count;
};

template <int PAIR, bool SHIFT, bool IMAGE>
__device__ __forceinline__ void interact(const ForceArgs &, const double4 pj, bool valid,
                                         double xi, double yi, double zi, double, double rl2,
                                         double sx, double sy, double sz, AccList &c, uint32_t j)
{
    double dx = IMAGE ? xi - (pj.x + sx) : xi - pj.x;
    double dy = IMAGE ? yi - (pj.y + sy) : yi - pj.y;
    double dz = IMAGE ? zi - (pj.z + sz) : zi - pj.z;
    double r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    if (valid && r2 < rl2) {
        if (c.count < c.cap) c.list[(int64_t)c.count * c.n + c.i] = j;
        c.count += 1;
    }
}

// One lane's particle.
struct Particle {
    int64_t i;      // sorted slot (a valid slot also for lanes without a particle)
    double x, y, z, rc, rc2;
};

// All candidates of one slot interval [jb, je) (empty for lanes without one), U loads in flight
// at a time; the particle itself is skipped. The loop runs until the wave's longest interval is
// done.
// Position record of slot j through the buffer descriptor of the position array: 32-bit byte
// offsets, and reads past the array's last record return zeros instead of touching memory.
template <int PAIR>
__device__ __forceinline__ double4 load_pos(__amdgpu_buffer_rsrc_t rs, uint32_t j)
{
    typedef double d2 __attribute__((ext_vector_type(2)));
    const d2 xy = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, j * 32u, 0, 0));
    double4 p;
    p.x = xy.x;
    p.y = xy.y;
    if (PAIR == DCM_PAIR_MAX) {
        const d2 zw = __builtin_bit_cast(d2, __builtin_amdgcn_raw_buffer_load_b128(rs, j * 32u + 16u, 0, 0));
        p.z = zw.x;
        p.w = zw.y;
    } else {
        p.z = __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(rs, j * 32u + 16u, 0, 0));
        p.w = 0.0;
    }
    return p;
}

template <int PAIR, bool SHIFT, bool IMAGE, int U, typename A>
__device__ __forceinline__ void scan(const ForceArgs &a, __amdgpu_buffer_rsrc_t rs, const Particle &q, uint32_t jb,
                                     uint32_t je, double sx, double sy, double sz, A &c)
{
    const uint32_t len = je - jb;
    for (uint32_t t = 0; __any(t < len); t += U) {
        double4 p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = load_pos<PAIR>(rs, jb + t + u);
#pragma unroll
        for (int u = 0; u < U; ++u)
            interact<PAIR, SHIFT, IMAGE>(a, p[u], t + u < len && jb + t + u != (uint32_t)q.i, q.x, q.y, q.z, q.rc,
                                         q.rc2, sx, sy, sz, c, jb + t + u);
    }
}

// The image variant runs only for waves in which some lane's interval is a periodic image.
template <int PAIR, bool SHIFT, int U, typename A>
__device__ __forceinline__ void scan_interval(const ForceArgs &a, __amdgpu_buffer_rsrc_t rs, const Particle &q,
                                              uint32_t jb, uint32_t je, double sx, double sy, double sz, A &c)
{
    const bool image = jb < je && (sx != 0.0 || sy != 0.0 || sz != 0.0);
    if (__any(image))
        scan<PAIR, SHIFT, true, U, A>(a, rs, q, jb, je, sx, sy, sz, c);
    else
        scan<PAIR, SHIFT, false, U, A>(a, rs, q, jb, je, sx, sy, sz, c);
}

// The slots of one force row that a wave's lanes scan, staged in LDS. Reading candidate
// positions lane by lane from global memory costs the vector-memory data path a cache line per
// lane and candidate (the lanes' windows are offset from each other), and that path, not the
// arithmetic, bounds the traversal. The wave instead loads the union of its lanes' x-intervals of
// a row once, coalesced, into LDS (coordinates in separate arrays, so that neighbouring lanes
// read neighbouring words), and the lanes read their candidates from there.
constexpr uint32_t kStageSlots = 192;
constexpr uint32_t kStagePad = 4;          // the candidate unroll reads up to U - 1 slots past
struct Stage {
    // z first: every array is then in reach of the LDS reads' immediate offsets from the
    // candidate's index scaled once per array
    double z[kStageSlots + kStagePad];
    double2 xy[kStageSlots + kStagePad];      // one 16-byte read per candidate
    double w[kStageSlots + kStagePad];
};

// SELF: some lane's own slot lies in its interval (only then is j != i tested).
// OVER: every lane's interval lies in one force row of the wave's window, so a lane may test the
// up to U - 1 slots after its interval's end in its last group of candidates: they hold
// particles of the same row beyond the lane's x-interval, hence out of range (the pair test
// decides them as it would anywhere), or, past the window's end, the stage's far sentinels. A lane
// past its interval reads only the sentinels at kStageSlots. No per-candidate window test is
// then needed.
template <int PAIR, bool SHIFT, bool IMAGE, bool SELF, bool OVER, int U, typename A>
__device__ __forceinline__ void scan_staged(const ForceArgs &a, const Stage &sg, uint32_t lo, const Particle &q,
                                            uint32_t jb, uint32_t je, double sx, double sy, double sz, A &c)
{
    const uint32_t len = je - jb;
    const uint32_t o = len ? jb - lo : 0u;
    // the particle's own slot as an offset into the interval (past its end if not in it)
    const uint32_t self = (uint32_t)q.i - jb;
    for (uint32_t t = 0; __any(t < len); t += U) {
        // one index per iteration; the stage has U - 1 slots of padding
        const uint32_t k = OVER ? (t < len ? o + t : kStageSlots) : min(o + t, kStageSlots);
        // byte offsets of slot k in the 8- and 16-byte arrays, each formed once (the opaque copy
        // keeps the compiler from deriving one from the other with extra instructions)
        uint32_t b8 = k * 8u;
        asm volatile("" : "+v"(b8));
        const uint32_t b16 = b8 + b8;
        const char *sb = reinterpret_cast<const char *>(&sg);
        const double *zs = reinterpret_cast<const double *>(sb + b8);
        const double2 *xys = reinterpret_cast<const double2 *>(sb + offsetof(Stage, xy) + b16);
        const double *ws = reinterpret_cast<const double *>(sb + offsetof(Stage, w) + b8);
        double4 p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double2 xy = xys[u];
            p[u].x = xy.x;
            p[u].y = xy.y;
            p[u].z = zs[u];
            p[u].w = PAIR == DCM_PAIR_MAX ? ws[u] : 0.0;
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
            interact<PAIR, SHIFT, IMAGE>(a, p[u], (OVER || t + u < len) && (!SELF || t + u != self), q.x, q.y,
                                         q.z, q.rc, q.rc2, sx, sy, sz, c, jb + t + u);
    }
}

// Wave-wide minimum / maximum with DPP lane moves (rows of 16 lanes by shifts, then row
// broadcasts; lane 63 ends with the result). Every lane of the wave must be active.
template <bool MAX>
__device__ __forceinline__ uint32_t wave_reduce_u(uint32_t v)
{
    const uint32_t id = MAX ? 0u : 0xFFFFFFFFu;
    auto op = [](uint32_t x, uint32_t y) { return MAX ? max(x, y) : min(x, y); };
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, 0x111, 0xf, 0xf, false));   // row_shr:1
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, 0x112, 0xf, 0xf, false));   // row_shr:2
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, 0x114, 0xf, 0xf, false));   // row_shr:4
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, 0x118, 0xf, 0xf, false));   // row_shr:8
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, 0x142, 0xa, 0xf, false));   // row_bcast:15
    v = op(v, (uint32_t)__builtin_amdgcn_update_dpp((int)id, (int)v, 0x143, 0xc, 0xf, false));   // row_bcast:31
    return (uint32_t)__builtin_amdgcn_readlane((int)v, 63);
}

__device__ __forceinline__ uint32_t wave_min_u(uint32_t v) { return wave_reduce_u<false>(v); }
__device__ __forceinline__ uint32_t wave_max_u(uint32_t v) { return wave_reduce_u<true>(v); }

// Slot range [jb, je) of every lane, from LDS when the lanes' ranges lie in one window of at
// most kStageSlots slots (the usual case: the wave's lanes share a force row), else directly.
// OVER as in scan_staged: the caller's lanes all scan one force row.
template <int PAIR, bool SHIFT, bool OVER, int U, typename A>
__device__ __forceinline__ void scan_row(const ForceArgs &a, __amdgpu_buffer_rsrc_t rs, Stage &sg, const Particle &q,
                                         uint32_t jb, uint32_t je, double sx, double sy, double sz, A &c)
{
    static_assert(U <= (int)kStagePad, "the candidate groups read up to U - 1 slots past the window");
    const bool has = jb < je;
    const uint32_t lo = wave_min_u(has ? jb : 0xFFFFFFFFu);
    const uint32_t hi = wave_max_u(has ? je : 0u);
    if (hi <= lo) return;
    if (hi - lo > kStageSlots) {
        scan_interval<PAIR, SHIFT, U, A>(a, rs, q, jb, je, sx, sy, sz, c);
        return;
    }
    const uint32_t lane = threadIdx.x & 63u;
    // the window's loads issued together (at most kStageSlots / 64 per lane), then stored
    constexpr int kStagePer = kStageSlots / 64;
    double4 pv[kStagePer];
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
        const uint32_t k = lane + 64u * u;
        pv[u] = load_pos<PAIR>(rs, lo + (k < hi - lo ? k : 0u));
    }
#pragma unroll
    for (int u = 0; u < kStagePer; ++u) {
        const uint32_t k = lane + 64u * u;
        if (k < hi - lo) {
            sg.xy[k] = make_double2(pv[u].x, pv[u].y + (OVER ? sy : 0.0));
            sg.z[k] = pv[u].z + (OVER ? sz : 0.0);
            if (PAIR == DCM_PAIR_MAX) sg.w[k] = pv[u].w;
        }
    }
    // far sentinels for the slots a lane's last group reads past the window's end
    if (OVER && lane < U - 1) sg.xy[hi - lo + lane].x = __builtin_inf();
    __syncthreads();
    // a single-row wave's image shift (uniform, none in x) is already in the staged coordinates:
    // the same sums the image form takes per candidate
    const bool image = !OVER && has && (sx != 0.0 || sy != 0.0 || sz != 0.0);
    const bool self = (uint32_t)q.i - jb < je - jb;
    if (__any(image))
        scan_staged<PAIR, SHIFT, true, true, OVER, U, A>(a, sg, lo, q, jb, je, sx, sy, sz, c);
    else if (__any(self))
        scan_staged<PAIR, SHIFT, false, true, OVER, U, A>(a, sg, lo, q, jb, je, sx, sy, sz, c);
    else
        scan_staged<PAIR, SHIFT, false, false, OVER, U, A>(a, sg, lo, q, jb, je, sx, sy, sz, c);
    __syncthreads();
}

__device__ __forceinline__ int wave_min(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = min(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

__device__ __forceinline__ int wave_max(int v)
{
    for (int off = 32; off > 0; off >>= 1) v = max(v, __shfl_xor(v, off, 64));
    return __builtin_amdgcn_readfirstlane(v);
}

// Walks the force rows (2^sz x 2^sy boxes in z and y, see cell_key) that come within particle
// i's search radius and scans, in each, the slot range of the x-interval the sphere cuts. The
// row loops are uniform over the wave: they run over the union of the lanes' row offsets
// relative to each lane's own force row, so lanes of one row look at the same neighbour rows
// together and their windows overlap. Each lane visits exactly its own rows, in increasing z,
// then y, then x.
// UNI: every live lane of the wave lies in one force row and no lane's x-interval can wrap
// around x, so row indices, their periodic wraps and image shifts are uniform over the wave
// (scalar) and each row is one slot range per lane.
template <int PAIR, bool SHIFT, int U, typename A, bool UNI>
__device__ __forceinline__ void traverse_rows(const ForceArgs &a, bool live, const Particle &q, double rs, int Yi,
                                              int Zi, A &c, Stage *sg)
{
    const Grid &g = a.grid;
    const double rs2 = rs * rs;
    const int nY = g.n[1] >> g.sy, nZ = g.n[2] >> g.sz, gs = g.sy + g.sz;
    const double Hy = g.h[1] * (double)(1 << g.sy), Hz = g.h[2] * (double)(1 << g.sz);
    // x-intervals are resolved in storage cells of h_x / 2^sx
    const double iHy = 1.0 / Hy, iHz = 1.0 / Hz, ihx = (double)(1 << g.sx) / g.h[0];
    const int ncx = g.n[0] << g.sx;
    const int zlo_r = live ? floor_mul(q.z - rs, iHz) - Zi : INT_MAX;
    const int zhi_r = live ? floor_mul(q.z + rs, iHz) - Zi : INT_MIN;
    const int zb = wave_min(zlo_r), ze = wave_max(zhi_r);
    // descriptor of the position array (gfx9 raw buffer; the record count is in bytes)
    const __amdgpu_buffer_rsrc_t pb =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.pos, 0, (int)((uint32_t)a.n * 32u), 0x00020000);
    for (int dZ = zb; dZ <= ze; ++dZ) {
        const int Z = Zi + dZ;
        const double zlo = Z * Hz;
        const double dzm = fmax(0.0, fmax(zlo - q.z, q.z - (zlo + Hz)));
        const double remz = rs2 - dzm * dzm;
        const bool zok = dZ >= zlo_r && dZ <= zhi_r && remz >= 0.0;
        int wZ = Z;
        double sz = 0.0;
        if (Z < 0) { wZ += nZ; sz = -g.L[2]; }
        else if (Z >= nZ) { wZ -= nZ; sz = g.L[2]; }
        const double ry = sqrt_up(zok ? remz : 0.0);
        const int ylo_r = zok ? floor_mul(q.y - ry, iHy) - Yi : INT_MAX;
        const int yhi_r = zok ? floor_mul(q.y + ry, iHy) - Yi : INT_MIN;
        const int yb = wave_min(ylo_r), ye = wave_max(yhi_r);
        for (int dY = yb; dY <= ye; ++dY) {
            const int Y = Yi + dY;
            const double ylo = Y * Hy;
            const double dym = fmax(0.0, fmax(ylo - q.y, q.y - (ylo + Hy)));
            const double rem = remz - dym * dym;
            const bool yok = zok && dY >= ylo_r && dY <= yhi_r && rem >= 0.0;
            int wY = Y;
            double sy = 0.0;
            if (Y < 0) { wY += nY; sy = -g.L[1]; }
            else if (Y >= nY) { wY -= nY; sy = g.L[1]; }
            const uint32_t row = (uint32_t)(wZ * nY + wY) * (uint32_t)ncx;
            // up to two contiguous slot ranges (the second one wraps around x)
            uint32_t b0 = 0, e0 = 0, b1 = 0, e1 = 0;
            double sx0 = 0.0, sx1 = 0.0;
            if (yok) {
                const double rx = sqrt_up(rem);
                const int ixlo = floor_mul(q.x - rx, ihx), ixhi = floor_mul(q.x + rx, ihx);
                int lo0 = ixlo, hi0 = ixhi, lo1 = 0, hi1 = -1;
                if (!UNI) {
                    if (ixlo < 0) {
                        lo0 = ixlo + ncx; hi0 = ncx - 1; sx0 = -g.L[0];
                        lo1 = 0; hi1 = ixhi;
                    } else if (ixhi >= ncx) {
                        hi0 = ncx - 1;
                        lo1 = 0; hi1 = ixhi - ncx; sx1 = g.L[0];
                    }
                }
                b0 = a.cell_start[(row + (uint32_t)lo0) << gs];
                e0 = a.cell_start[(row + (uint32_t)hi0 + 1u) << gs];
                if (!UNI && hi1 >= lo1) {
                    b1 = a.cell_start[(row + (uint32_t)lo1) << gs];
                    e1 = a.cell_start[(row + (uint32_t)hi1 + 1u) << gs];
                }
            }
            if (sg) scan_row<PAIR, SHIFT, UNI, U, A>(a, pb, *sg, q, b0, e0, sx0, sy, sz, c);
            else scan_interval<PAIR, SHIFT, U, A>(a, pb, q, b0, e0, sx0, sy, sz, c);
            if (!UNI && __any(b1 < e1)) scan_interval<PAIR, SHIFT, U, A>(a, pb, q, b1, e1, sx1, sy, sz, c);
        }
    }
}

template <int PAIR, bool SHIFT, int U, typename A>
__device__ __forceinline__ void traverse(const ForceArgs &a, bool live, const Particle &q, double rc_max, A &c,
                                         Stage *sg = nullptr)
{
    const Grid &g = a.grid;
    // search radius (slightly enlarged so that rounding in the box bounds never drops a box
    // that holds an in-range particle; the pair test itself is exact)
    double rs = PAIR == DCM_PAIR_MAX ? rc_max : q.rc;
    rs = rs * (1.0 + 1e-12) + 1e-9;
    const double iHy = 1.0 / (g.h[1] * (double)(1 << g.sy)), iHz = 1.0 / (g.h[2] * (double)(1 << g.sz));
    const int Yi = live ? floor_mul(q.y, iHy) : 0, Zi = live ? floor_mul(q.z, iHz) : 0;
    // one force row for every live lane, and every x-interval inside [0, L_x)
    const int ylo = wave_min(live ? Yi : INT_MAX), yhi = wave_max(live ? Yi : INT_MIN);
    const int zlo = wave_min(live ? Zi : INT_MAX), zhi = wave_max(live ? Zi : INT_MIN);
    // (with the largest x reach a row's interval can take, so that no interval leaves [0, L_x))
    const double rsx = x_reach(rs);
    const bool inside = !live || (q.x - rsx >= 0.0 && q.x + rsx <= g.L[0] * (1.0 - 1e-9));
    if (ylo == yhi && zlo == zhi && __all(inside))
        traverse_rows<PAIR, SHIFT, U, A, true>(a, live, q, rs, ylo, zlo, c, sg);
    else
        traverse_rows<PAIR, SHIFT, U, A, false>(a, live, q, rs, Yi, Zi, c, sg);
}

// The candidates of lane i's list, U at a time, until the wave's longest list is done. The
// periodic image of x_j is the one nearest x_i (shift +L where x_i - x_j > L / 2, -L below
// -L / 2), so dx = x_i - (x_j + shift) is the number the cell traversal and the minimum-image
// convention give for every pair within r_c < L / 2.
template <bool SHIFT, int U, typename A>
__device__ __forceinline__ void list_scan(const ForceArgs &a, bool live, const Particle &q, A &c)
{
    const Grid &g = a.grid;
    const uint32_t cnt = live ? a.nlist[q.i] : 0u;
    const int kmax = wave_max((int)cnt);
    const __amdgpu_buffer_rsrc_t pb =
        __builtin_amdgcn_make_buffer_rsrc((void *)a.pos, 0, (int)((uint32_t)a.n * 32u), 0x00020000);
    const double hx = 0.5 * g.L[0], hy = 0.5 * g.L[1], hz = 0.5 * g.L[2];
    for (int k = 0; k < kmax; k += U) {
        uint32_t jj[U];
#pragma unroll
        for (int u = 0; u < U; ++u)
            jj[u] = (uint32_t)(k + u) < cnt ? a.list[(int64_t)(k + u) * a.n + q.i] : (uint32_t)q.i;
        double4 p[U];
#pragma unroll
        for (int u = 0; u < U; ++u) p[u] = load_pos<DCM_PAIR_I>(pb, jj[u]);
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double ex = q.x - p[u].x, ey = q.y - p[u].y, ez = q.z - p[u].z;
            const double sx = ex > hx ? g.L[0] : (ex < -hx ? -g.L[0] : 0.0);
            const double sy = ey > hy ? g.L[1] : (ey < -hy ? -g.L[1] : 0.0);
            const double sz = ez > hz ? g.L[2] : (ez < -hz ? -g.L[2] : 0.0);
            interact<DCM_PAIR_I, SHIFT, true>(a, p[u], (uint32_t)(k + u) < cnt, q.x, q.y, q.z, q.rc, q.rc2, sx, sy,
                                              sz, c, jj[u]);
        }
    }
}

// Duration class, 16 per octave (monotone in t), numbered from the longest: 0 .. 511.
__device__ __forceinline__ uint32_t duration_class(uint32_t t)
{
    const uint32_t v = t < 0xffffffffu ? t + 1u : t;
    const int e = 31 - __clz(v);
    const uint32_t c = e < 4 ? v : ((uint32_t)(e - 3) << 4) | ((v >> (e - 4)) & 15u);
    return 511u - (c < 511u ? c : 511u);
}

constexpr int kWaveClasses = 512;
constexpr int kWaveGroups = 64;

__device__ __forceinline__ void wave_chunk(uint32_t nb, uint32_t w, uint32_t &lo, uint32_t &hi)
{
    const uint32_t per = (nb + kWaveGroups - 1) / kWaveGroups;
    lo = min(nb, w * per);
    hi = min(nb, lo + per);
}

// Compiled for 4 waves per SIMD (128 VGPRs per lane).
template <int PAIR, bool SHIFT, int U, int PREC, bool LIST = false>
struct KForces {
    static constexpr int kThreads = kForceBlock, kWaves = 4;
    struct Args {
        ForceArgs a;
        double rc_max;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t);
};

template <int PAIR, bool SHIFT, int U, int PREC, bool LIST>
__device__ void KForces<PAIR, SHIFT, U, PREC, LIST>::run(const Args &args_, uint32_t blk, uint32_t nblk)
{
    const ForceArgs &a = args_.a;
    const double rc_max = args_.rc_max;
    // the wave this workgroup takes: longest (in the last launch) first, so that the waves
    // still running at the end are short ones; the hardware deals workgroups round-robin over
    // the XCDs, which spreads every duration class over all of them
    const int64_t b = a.order ? (int64_t)min(a.order[blk], nblk - 1u) : (int64_t)blk;
    const uint64_t t_start = __builtin_amdgcn_s_memrealtime();
    const int64_t i = b * kForceBlock + threadIdx.x;
    const bool have = i < a.n;
    Particle q;
    q.i = have ? i : 0;
    const double4 pi = a.pos[q.i];
    q.x = pi.x;
    q.y = pi.y;
    q.z = pi.z;
    q.rc = pi.w;
    q.rc2 = q.rc * q.rc;
    // a non-finite position or a cutoff outside (0, rc_max] would send the box loops out of the
    // grid: such a particle gets no traversal and a NaN force (flagged below)
    const bool sane = isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && q.rc > 0.0 && q.rc <= rc_max;
    const bool live = have && sane;
    // every lane of the wave takes part in the (wave-uniform) traversal
    typedef Acc AccT;
    AccT c = {};
    Stage *stage = nullptr;
    if constexpr (!LIST) {
        __shared__ Stage st;
        stage = &st;
        // the padding slots stay far sentinels (x = +inf: never in range) for the whole launch
        if (threadIdx.x < kStagePad) st.xy[kStageSlots + threadIdx.x].x = __builtin_inf();
    }
    if (PREC == DCM_FP64) {
        if (LIST) list_scan<SHIFT, U, AccT>(a, live, q, c);
        else traverse<PAIR, SHIFT, U, AccT>(a, live, q, rc_max, c, stage);
        // the pair loop's units (see Acc): forces and virial times 24 eps sigma^6; sum
        // ((sigma/r)^12 - (sigma/r)^6) from the virial trace and the sum of r^-6
        const double esum = 0.5 * (0.5 * a.sigma6x2) * ((c.wxx + c.wyy + c.wzz) - c.e);
        c.fx *= a.eps24s6; c.fy *= a.eps24s6; c.fz *= a.eps24s6;
        c.wxx *= a.eps24s6; c.wyy *= a.eps24s6; c.wzz *= a.eps24s6;
        c.wxy *= a.eps24s6; c.wxz *= a.eps24s6; c.wyz *= a.eps24s6;
        c.e = esum;
    } else {
        Acc32 c32 = {};
        if (LIST) list_scan<SHIFT, U, Acc32>(a, live, q, c32);
        else traverse<PAIR, SHIFT, U, Acc32>(a, live, q, rc_max, c32, stage);
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
    if (have) {
        const double rc2 = q.rc2;
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
        if (a.wave_time) {
            const uint64_t dt = __builtin_amdgcn_s_memrealtime() - t_start;
            const uint32_t t32 = dt < 0xffffffffull ? (uint32_t)dt : 0xffffffffu;
            a.wave_time[b] = t32;
            // the count of the ordering's counting sort: chunk of this wave, duration class
            if (a.wave_hist) {
                const uint32_t per = (nblk + kWaveGroups - 1) / kWaveGroups;
                atomicAdd(&a.wave_hist[(uint32_t)b / per * kWaveClasses + duration_class(t32)], 1u);
            }
        }
    }
}

// Counting sort of the waves by duration class, longest first, over kWaveGroups chunks of
// consecutive waves: per-chunk class counts (taken by the force kernel's waves as they finish,
// or by KWaveCount), the start of every (class, chunk) pair, and the scatter, which leaves the
// counts at zero for the next force launch. Waves of one class and chunk take no fixed order
// among themselves.
struct KWaveCount {
    static constexpr int kThreads = 256, kWaves = 0;
    struct Args {
        const uint32_t *t;
        uint32_t *hist;     // [kWaveGroups][kWaveClasses]
        uint32_t nb;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        __shared__ uint32_t cnt[kWaveClasses];
        for (int k = threadIdx.x; k < kWaveClasses; k += kThreads) cnt[k] = 0u;
        __syncthreads();
        uint32_t lo, hi;
        wave_chunk(a.nb, blk, lo, hi);
        for (uint32_t k = lo + threadIdx.x; k < hi; k += kThreads) atomicAdd(&cnt[duration_class(a.t[k])], 1u);
        __syncthreads();
        for (int k = threadIdx.x; k < kWaveClasses; k += kThreads) a.hist[blk * kWaveClasses + k] = cnt[k];
    }
};

// hist[w][c] becomes the first slot of class c's waves from chunk w: the waves of all longer
// classes, then those of class c in earlier chunks.
struct KWaveStarts {
    static constexpr int kThreads = kWaveClasses, kWaves = 0;
    struct Args { uint32_t *hist; };
    static __device__ void run(const Args &a, uint32_t, uint32_t)
    {
        __shared__ uint32_t tot[2][kWaveClasses];
        const int c = threadIdx.x;
        uint32_t sum = 0u;
        for (int w = 0; w < kWaveGroups; ++w) sum += a.hist[w * kWaveClasses + c];
        tot[0][c] = sum;
        __syncthreads();
        // inclusive sums over the classes: Hillis-Steele doubling steps, ping-ponging
        int src = 0;
        for (int off = 1; off < kWaveClasses; off <<= 1) {
            tot[1 - src][c] = tot[src][c] + (c >= off ? tot[src][c - off] : 0u);
            __syncthreads();
            src = 1 - src;
        }
        uint32_t base = c > 0 ? tot[src][c - 1] : 0u;
        for (int w = 0; w < kWaveGroups; ++w) {
            const uint32_t h = a.hist[w * kWaveClasses + c];
            a.hist[w * kWaveClasses + c] = base;
            base += h;
        }
    }
};

struct KWaveScatter {
    static constexpr int kThreads = 256, kWaves = 0;
    struct Args {
        const uint32_t *t;
        uint32_t *hist;
        uint32_t *order;
        uint32_t nb;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        __shared__ uint32_t next[kWaveClasses];
        for (int k = threadIdx.x; k < kWaveClasses; k += kThreads) {
            next[k] = a.hist[blk * kWaveClasses + k];
            a.hist[blk * kWaveClasses + k] = 0u;
        }
        __syncthreads();
        uint32_t lo, hi;
        wave_chunk(a.nb, blk, lo, hi);
        for (uint32_t k = lo + threadIdx.x; k < hi; k += kThreads)
            a.order[atomicAdd(&next[duration_class(a.t[k])], 1u)] = k;
    }
};

// Neighbour lists: the force kernel's traversal with the search radius r_c[i] + skin, each
// slot within it recorded (Alg. 3.3's list of the pairs within r_c + r_s).
struct KBuildList {
    static constexpr int kThreads = kForceBlock, kWaves = 4;
    struct Args {
        ForceArgs a;
        double skin;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t);
};

__device__ void KBuildList::run(const Args &args_, uint32_t blk, uint32_t)
{
    const ForceArgs &a = args_.a;
    const int64_t i = (int64_t)blk * kForceBlock + threadIdx.x;
    const bool have = i < a.n;
    Particle q;
    q.i = have ? i : 0;
    const double4 pi = a.pos[q.i];
    q.x = pi.x;
    q.y = pi.y;
    q.z = pi.z;
    q.rc = pi.w + args_.skin;
    q.rc2 = q.rc * q.rc;
    const bool sane = isfinite(q.x) && isfinite(q.y) && isfinite(q.z) && pi.w > 0.0 && pi.w <= a.rc_max;
    AccList c = {a.list, a.n, i, a.list_cap, 0u};
    traverse<DCM_PAIR_I, false, 4, AccList>(a, have && sane, q, a.rc_max, c);
    if (have) {
        a.nlist[i] = c.count < a.list_cap ? c.count : a.list_cap;
        if (c.count > a.list_cap) atomicOr(a.flags, kFlagListOverflow);
    }
}

}  // namespace

int force_blocks(int64_t n) { return (int)((n + kForceBlock - 1) / kForceBlock); }

template <int PREC>
static void launch_prec(const ForceArgs &a, int nb, hipStream_t st)
{
    constexpr int U = 4;
    const uint32_t blocks = (uint32_t)nb;
    if (a.list_mode) {
        if (a.energy_shift) emit<KForces<DCM_PAIR_I, true, U, PREC, true>>({a, a.rc_max}, blocks, st);
        else emit<KForces<DCM_PAIR_I, false, U, PREC, true>>({a, a.rc_max}, blocks, st);
        return;
    }
    if (a.pair_rule == DCM_PAIR_MAX) {
        if (a.energy_shift) emit<KForces<DCM_PAIR_MAX, true, U, PREC>>({a, a.rc_max}, blocks, st);
        else emit<KForces<DCM_PAIR_MAX, false, U, PREC>>({a, a.rc_max}, blocks, st);
    } else {
        if (a.energy_shift) emit<KForces<DCM_PAIR_I, true, U, PREC>>({a, a.rc_max}, blocks, st);
        else emit<KForces<DCM_PAIR_I, false, U, PREC>>({a, a.rc_max}, blocks, st);
    }
}

void launch_build_list(const ForceArgs &a, double skin, hipStream_t st)
{
    emit<KBuildList>({a, skin}, (uint32_t)force_blocks(a.n), st);
}

size_t wave_order_scratch_words() { return (size_t)kWaveGroups * kWaveClasses; }

void launch_wave_order(const uint32_t *wave_time, uint32_t *order, uint32_t *hist, int64_t nb, bool counted,
                       hipStream_t st)
{
    if (!counted) emit<KWaveCount>({wave_time, hist, (uint32_t)nb}, kWaveGroups, st);
    emit<KWaveStarts>({hist}, 1, st);
    emit<KWaveScatter>({wave_time, hist, order, (uint32_t)nb}, kWaveGroups, st);
}

void launch_forces(const ForceArgs &a, hipStream_t st)
{
    const int nb = force_blocks(a.n);
    if (a.precision == DCM_FP32C) launch_prec<DCM_FP32C>(a, nb, st);
    else launch_prec<DCM_FP64>(a, nb, st);
}

void launch_force_wave_order(const ForceArgs &a, hipStream_t st)
{
    if (a.order && a.wave_time) launch_wave_order(a.wave_time, a.order, a.wave_hist, force_blocks(a.n), true, st);
}

}  // namespace dcm
