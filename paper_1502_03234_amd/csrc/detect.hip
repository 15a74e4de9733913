// detect.hip -- interface detection on the box grid (Section 4, Fig. 14).
//
//   smoothing        periodic [1,2,1] per axis on the counts of Eq. 9 (integer, exact)
//   two-means        Eq. 14 with K = 2: histogram of the smoothed values, then Lloyd's
//                    iteration from (min, max) in one workgroup with exact integer sums
//   labels           Eq. 11-12: liquid (0) iff value > threshold, else vapor (1)
//   components       Section 4.2: 6-connected periodic components by lock-free union-find
//                    (links always point to the smaller index, so each component ends up
//                    named by its smallest box index); components below the size limit
//                    flip phase, vapor first, then liquid on the updated image
//   distance         Eq. 15-19 and Section 4.3.2: in-place Godunov relaxation of the liquid
//                    boxes, keeping only values inside the band r_c^max + h, repeated until a
//                    sweep changes nothing
//   cutoffs          Alg. 3.1 trilinear interpolation of box-centre distances, then Eq. 7-8
#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

inline unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ __forceinline__ int64_t lin(const Grid &g, int64_t i, int64_t j, int64_t k)
{
    return (k * g.n[1] + j) * g.n[0] + i;
}

// Box coordinates of linear index c. Grids hold fewer than 2^31 boxes (checked when a system
// or a grid workspace is set up), so 32-bit unsigned division suffices (64-bit division is a
// long emulated sequence).
__device__ __forceinline__ void coords(const Grid &g, int64_t c, int64_t &i, int64_t &j, int64_t &k)
{
    const uint32_t u = (uint32_t)c, nx = (uint32_t)g.n[0], ny = (uint32_t)g.n[1];
    const uint32_t r = u / nx;
    const uint32_t z = r / ny;
    i = (int64_t)(u - r * nx);
    j = (int64_t)(r - z * ny);
    k = (int64_t)z;
}

// ---- smoothing ------------------------------------------------------------------------
// One smoothing pass, [1, 2, 1] along x, then y, then z, periodic, on a 32 x 8 x 4 block of boxes
// staged in LDS with a one-box halo. The sums are integers, so doing the three axes per block
// gives the same values as three whole-grid passes.
constexpr int SX = 32, SY = 8, SZ = 4;

struct KSmooth3 {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        const uint32_t *in;
        uint32_t *out;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

// v in [-1, 2n): periodic index; axes shorter than a block (v past 2n - 1) take the remainder.
__device__ __forceinline__ int wrap_halo(int v, int n)
{
    if (v < 0) return v + n;
    if (v < n) return v;
    v -= n;
    return v < n ? v : v % n;
}

__device__ void KSmooth3::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    const uint32_t *in = args_.in;
    __shared__ uint32_t A[SZ + 2][SY + 2][SX + 2];
    __shared__ uint32_t B[SZ + 2][SY + 2][SX];
    __shared__ uint32_t C[SZ + 2][SY][SX];
    const int ntx = (g.n[0] + SX - 1) / SX, nty = (g.n[1] + SY - 1) / SY;
    const int x0 = (int)(blk % ntx) * SX, y0 = (int)((blk / ntx) % nty) * SY, z0 = (int)(blk / (ntx * nty)) * SZ;
    // positions past the grid's far edge hold wrapped values too; only in-grid boxes are written.
    // A thread's loads are all in flight at once (one round trip, not one per load).
    constexpr int kHalo = (SZ + 2) * (SY + 2) * (SX + 2);
    constexpr int kHaloPer = (kHalo + kBlock - 1) / kBlock;
    uint32_t hv[kHaloPer];
#pragma unroll
    for (int it = 0; it < kHaloPer; ++it) {
        const int q = (int)threadIdx.x + it * kBlock;
        const int qq = q < kHalo ? q : 0;
        const int hx = qq % (SX + 2), hy = (qq / (SX + 2)) % (SY + 2), hz = qq / ((SX + 2) * (SY + 2));
        // periodic neighbours without a division (block origins lie inside the grid)
        const int gx = wrap_halo(x0 + hx - 1, g.n[0]);
        const int gy = wrap_halo(y0 + hy - 1, g.n[1]);
        const int gz = wrap_halo(z0 + hz - 1, g.n[2]);
        hv[it] = in[((int64_t)gz * g.n[1] + gy) * g.n[0] + gx];
    }
#pragma unroll
    for (int it = 0; it < kHaloPer; ++it) {
        const int q = (int)threadIdx.x + it * kBlock;
        if (q < kHalo) A[q / ((SX + 2) * (SY + 2))][(q / (SX + 2)) % (SY + 2)][q % (SX + 2)] = hv[it];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < (SZ + 2) * (SY + 2) * SX; q += kBlock) {
        const int x = q % SX, y = (q / SX) % (SY + 2), z = q / (SX * (SY + 2));
        B[z][y][x] = A[z][y][x] + 2u * A[z][y][x + 1] + A[z][y][x + 2];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < (SZ + 2) * SY * SX; q += kBlock) {
        const int x = q % SX, y = (q / SX) % SY, z = q / (SX * SY);
        C[z][y][x] = B[z][y][x] + 2u * B[z][y + 1][x] + B[z][y + 2][x];
    }
    __syncthreads();
    for (int q = threadIdx.x; q < SZ * SY * SX; q += kBlock) {
        const int x = q % SX, y = (q / SX) % SY, z = q / (SX * SY);
        const int gx = x0 + x, gy = y0 + y, gz = z0 + z;
        if (gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) continue;
        args_.out[lin(g, gx, gy, gz)] = C[z][y][x] + 2u * C[z + 1][y][x] + C[z + 2][y][x];
    }
}

struct KCountFromRanges {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        const uint32_t *cell_start;
        uint32_t *out;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

// Threads take the boxes in storage order (force row, then x, then the box's place in its row),
// so that neighbouring threads read neighbouring cell starts; the image is written in box order.
__device__ void KCountFromRanges::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    const uint32_t *cell_start = args_.cell_start;
    const int64_t t = (int64_t)blk * blockDim.x + threadIdx.x;
    if (t >= g.G) return;
    const int sub_bits = g.sy + g.sz;
    const uint32_t sub = (uint32_t)t & ((1u << sub_bits) - 1u);
    const uint32_t rest = (uint32_t)(t >> sub_bits);
    const uint32_t a = rest % (uint32_t)g.n[0];
    const uint32_t row = rest / (uint32_t)g.n[0];
    const uint32_t rows_y = (uint32_t)g.n[1] >> g.sy;
    const uint32_t b = ((row % rows_y) << g.sy) | (sub & ((1u << g.sy) - 1u));
    const uint32_t c = ((row / rows_y) << g.sz) | (sub >> g.sy);
    args_.out[((int64_t)c * g.n[1] + b) * g.n[0] + a] = box_count(g, cell_start, (int32_t)a, (int32_t)b, (int32_t)c);
}

// ---- histogram and two-means ----------------------------------------------------------
constexpr int kLdsBins = 8192;

struct KHist {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        const uint32_t *img;
        int64_t G;
        uint32_t *hist;
        uint32_t *flags;
        int aligned;        // img is 16-byte aligned (a caller's image need not be)
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KHist::run(const Args &args_, uint32_t blk, uint32_t nblk)
{
    const uint32_t *img = args_.img;
    int64_t G = args_.G;
    uint32_t *hist = args_.hist;
    uint32_t *flags = args_.flags;
    __shared__ uint32_t lh[kLdsBins];
    for (int b = threadIdx.x; b < kLdsBins; b += kBlock) lh[b] = 0;
    __syncthreads();
    // empty boxes (most of the vapor) are counted in a register: the zero bin would otherwise
    // take most of the LDS atomics, all on one address
    uint32_t zeros = 0;
    auto add = [&](uint32_t v) {
        if (v == 0u) ++zeros;
        else if (v < (uint32_t)kLdsBins) atomicAdd(&lh[v], 1u);
        else if (v < (uint32_t)kHistBins) atomicAdd(&hist[v], 1u);
        else atomicOr(flags, kFlagHistOverflow);
    };
    // four boxes per 16-byte load where the image is aligned, then the last G % 4
    const int64_t G4 = args_.aligned ? G / 4 : 0;
    const int64_t t0 = (int64_t)blk * blockDim.x + threadIdx.x, stride = (int64_t)nblk * blockDim.x;
    // four 16-byte loads in flight per thread and round
    for (int64_t q = t0; q < G4; q += 4 * stride) {
        uint4 w[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            const int64_t qu = q + u * stride;
            w[u] = ((const uint4 *)img)[qu < G4 ? qu : q];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
            if (q + u * stride < G4) {
                add(w[u].x);
                add(w[u].y);
                add(w[u].z);
                add(w[u].w);
            }
    }
    for (int64_t c = 4 * G4 + t0; c < G; c += stride) add(img[c]);
    for (int off = 32; off > 0; off >>= 1) zeros += __shfl_xor(zeros, off, 64);
    if ((threadIdx.x & 63) == 0 && zeros) atomicAdd(&lh[0], zeros);
    __syncthreads();
    for (int b = threadIdx.x; b < kLdsBins; b += kBlock)
        if (lh[b]) atomicAdd(&hist[b], lh[b]);
}

constexpr int kTmThreads = 1024;

// Two-means on the histogram: the occupied range [min, max] is found by the whole block, copied
// to LDS, and the Lloyd iterations then run in one wave with shuffle reductions only. All sums
// are exact integers, so their order does not matter. The histogram is left at zero for the
// next detection.
constexpr int kTmLds = 16384;

struct KTwoMeans {
    static constexpr int kThreads = kTmThreads, kWaves = 0;
    struct Args {
        uint32_t *hist;
        double *km;
        long long *stats_iter;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KTwoMeans::run(const Args &args_, uint32_t, uint32_t)
{
    uint32_t *hist = args_.hist;
    double *km = args_.km;
    long long *stats_iter = args_.stats_iter;
    __shared__ int lmn[16], lmx[16];
    __shared__ uint32_t lh[kTmLds];
    const int tid = threadIdx.x, w = tid >> 6;
    int mn = kHistBins, mx = -1;
    static_assert(kHistBins % (4 * kTmThreads) == 0, "whole uint4 loads");
    // a fixed count, unrolled, so that a thread's 16 loads are in flight together rather than
    // one at a time
#pragma unroll
    for (int qq = 0; qq < kHistBins / (4 * kTmThreads); ++qq) {
        const int b0 = 4 * tid + qq * 4 * kTmThreads;
        const uint4 v = *reinterpret_cast<const uint4 *>(hist + b0);
        const uint32_t h[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
        for (int q = 0; q < 4; ++q)
            if (h[q]) { mn = min(mn, b0 + q); mx = max(mx, b0 + q); }
    }
    for (int off = 32; off > 0; off >>= 1) {
        mn = min(mn, __shfl_xor(mn, off, 64));
        mx = max(mx, __shfl_xor(mx, off, 64));
    }
    if ((tid & 63) == 0) { lmn[w] = mn; lmx[w] = mx; }
    __syncthreads();
    mn = kHistBins; mx = -1;
    for (int q = 0; q < 16; ++q) { mn = min(mn, lmn[q]); mx = max(mx, lmx[q]); }
    if (mx < 0) mn = mx = 0;                    // empty histogram (cannot happen for G >= 27)
    const bool staged = mx - mn + 1 <= kTmLds;
    if (staged) {
        for (int b = mn + tid; b <= mx; b += kTmThreads) {
            lh[b - mn] = hist[b];
            hist[b] = 0u;
        }
    }
    __syncthreads();
    if (w != 0) return;
    if (mn == mx) {
        if (tid == 0) {
            km[0] = (double)mn; km[1] = (double)mx; km[2] = (double)mn - 1.0;
            if (stats_iter) *stats_iter = 0;
        }
        return;
    }
    double cv = (double)mn, cl = (double)mx;
    long long prev = -1;
    int it;
    for (it = 1; it <= 1000; ++it) {
        const double m = 0.5 * (cv + cl);
        long long sv = 0, nv = 0, sl = 0, nl = 0;
        for (int b = mn + tid; b <= mx; b += 64) {
            const long long c = staged ? lh[b - mn] : hist[b];
            if ((double)b > m) { sl += c * b; nl += c; }
            else               { sv += c * b; nv += c; }
        }
        for (int off = 32; off > 0; off >>= 1) {
            sv += __shfl_xor(sv, off, 64);
            nv += __shfl_xor(nv, off, 64);
            sl += __shfl_xor(sl, off, 64);
            nl += __shfl_xor(nl, off, 64);
        }
        cv = (double)sv / (double)nv;
        cl = (double)sl / (double)nl;
        if (nl == prev) break;
        prev = nl;
    }
    if (!staged)
        for (int b = mn + tid; b <= mx; b += 64) hist[b] = 0u;
    if (tid == 0) {
        km[0] = cv; km[1] = cl; km[2] = 0.5 * (cv + cl);
        if (stats_iter) *stats_iter = it;
    }
}

// ---- labels and components ------------------------------------------------------------
struct KThreshold {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        const uint32_t *img;
        const double *km;
        int64_t G;
        uint8_t *raw;
        uint8_t *label;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KThreshold::run(const Args &args_, uint32_t blk, uint32_t)
{
    const uint32_t *img = args_.img;
    const double *km = args_.km;
    int64_t G = args_.G;
    uint8_t *raw = args_.raw;
    uint8_t *label = args_.label;
    int64_t c = (int64_t)blk * blockDim.x + threadIdx.x;
    if (c >= G) return;
    uint8_t s = ((double)img[c] > km[2]) ? 0 : 1;
    raw[c] = s;
    label[c] = s;
}

__device__ __forceinline__ uint32_t load_parent(uint32_t *parent, uint32_t x)
{
    return __hip_atomic_load(parent + x, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void store_parent(uint32_t *parent, uint32_t x, uint32_t v)
{
    __hip_atomic_store(parent + x, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Root of x's tree with path halving: every visited box is re-pointed at its grandparent.
// Parents only ever decrease along a tree path, so the plain stores keep the forest valid
// whatever other threads do concurrently.
__device__ uint32_t find_root(uint32_t *parent, uint32_t x)
{
    uint32_t p = load_parent(parent, x);
    while (p != x) {
        uint32_t gp = load_parent(parent, p);
        if (gp != p) store_parent(parent, x, gp);
        x = p;
        p = gp;
    }
    return x;
}

// Join the trees of a and b; the larger root is linked under the smaller one.
__device__ void unite(uint32_t *parent, uint32_t a, uint32_t b)
{
    for (;;) {
        a = find_root(parent, a);
        b = find_root(parent, b);
        if (a == b) return;
        if (a < b) { uint32_t t = a; a = b; b = t; }
        uint32_t old = atomicMin(parent + a, b);
        if (old == a) return;
        a = old;
    }
}

// Block-local labelling: each workgroup owns a CT^3 tile of boxes and records the tile's kind.
// A tile without boxes of the phase, or made only of them with at least `limit` in the grid (one
// piece, large whatever it joins), writes nothing else. Any other tile joins same-phase face
// neighbours with a union-find in LDS and writes for every box of the phase the global index of
// its tile-local root (the smallest member of its tile-local piece: local and global linear
// orders agree inside a tile) and the piece's size; csize is cleared on the way for the boxes of
// the phase (the only boxes that can be roots).
constexpr int CT = 8;
constexpr int kCtBoxes = CT * CT * CT;

__device__ __forceinline__ uint32_t lfind(uint32_t *lp, uint32_t x)
{
    uint32_t p = lp[x];
    while (p != x) {
        uint32_t gp = lp[p];
        if (gp != p) lp[x] = gp;
        x = p;
        p = gp;
    }
    return x;
}

__device__ __forceinline__ void lunite(uint32_t *lp, uint32_t a, uint32_t b)
{
    for (;;) {
        a = lfind(lp, a);
        b = lfind(lp, b);
        if (a == b) return;
        if (a < b) { uint32_t t = a; a = b; b = t; }
        uint32_t old = atomicMin(lp + a, b);
        if (old == a) return;
        a = old;
    }
}

// Tile kinds of one component pass (ctile[t]): kCtFull tiles keep per-box union-find entries;
// a kCtLarge tile holds only boxes of the phase, at least `limit` of them (one piece that is large
// whatever it joins); a kCtNone tile holds no box of the phase. Per-box entries of the last two
// kinds are neither written nor read.
constexpr uint8_t kCtFull = 0, kCtLarge = 1, kCtNone = 2;

__device__ __forceinline__ int64_t ct_tile(const Grid &g, int64_t i, int64_t j, int64_t k)
{
    const int64_t ntx = (g.n[0] + CT - 1) / CT, nty = (g.n[1] + CT - 1) / CT;
    return ((k / CT) * nty + j / CT) * ntx + i / CT;
}

// Box q (0 .. CT^3 - 1, x fastest) of component tile t, if it lies inside the grid.
__device__ __forceinline__ bool ct_box(const Grid &g, int64_t t, int q, int64_t &c)
{
    const int64_t ntx = (g.n[0] + CT - 1) / CT, nty = (g.n[1] + CT - 1) / CT;
    const int64_t i = (t % ntx) * CT + q % CT, j = ((t / ntx) % nty) * CT + (q / CT) % CT;
    const int64_t k = (t / (ntx * nty)) * CT + q / (CT * CT);
    if (i >= g.n[0] || j >= g.n[1] || k >= g.n[2]) return false;
    c = lin(g, i, j, k);
    return true;
}

// The per-box kernels after the merge run one workgroup per component tile: only boxes of
// kCtFull tiles hold union-find entries, so the other tiles' workgroups exit at once.
constexpr int kCtPer = CT * CT * CT / kBlock;      // boxes per thread

// Tile kinds first, one wave per tile: each lane counts the in-grid boxes and the boxes of the
// phase in one x-row of 8 boxes (one 8-byte load where the row is whole and aligned).
struct KCcClassify {
    static constexpr int kThreads = 64, kWaves = 0;
    struct Args {
        Grid g;
        const uint8_t *label;
        uint8_t phase;
        uint8_t *ctile;
        uint32_t limit;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

static_assert(CT == 8 && CT * CT == 64, "one lane per x-row of a component tile");

__device__ void KCcClassify::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    const uint8_t *label = args_.label;
    const uint8_t phase = args_.phase;
    const int ntx = (g.n[0] + CT - 1) / CT, nty = (g.n[1] + CT - 1) / CT;
    const int b = blk;
    const int x0 = (b % ntx) * CT, y0 = ((b / ntx) % nty) * CT, z0 = (b / (ntx * nty)) * CT;
    const int l = threadIdx.x;
    const int gy = y0 + l % CT, gz = z0 + l / CT;
    int nin = 0, nmine = 0;
    if (gy < g.n[1] && gz < g.n[2]) {
        const int64_t c0 = lin(g, x0, gy, gz);
        const int nx = min(CT, (int)g.n[0] - x0);
        // (labels may be a caller's buffer at any byte offset: the address itself is checked)
        if (nx == CT && ((uintptr_t)(label + c0) & 7u) == 0) {
            // labels are 0 or 1: the byte sum of the row counts the liquid boxes
            const uint64_t w = *reinterpret_cast<const uint64_t *>(label + c0);
            const int ones = __popcll(w & 0x0101010101010101ull);
            nin = CT;
            nmine = phase ? ones : CT - ones;
        } else {
            nin = nx;
            for (int x = 0; x < nx; ++x) nmine += label[c0 + x] == phase;
        }
    }
    for (int off = 32; off > 0; off >>= 1) {
        nin += __shfl_xor(nin, off, 64);
        nmine += __shfl_xor(nmine, off, 64);
    }
    if (l == 0) {
        uint8_t kind = kCtFull;
        if (nmine == 0) kind = kCtNone;
        else if (nmine == nin && (uint32_t)nmine >= args_.limit) kind = kCtLarge;
        args_.ctile[b] = kind;
    }
}

// The union-find runs on the tiles of kind kCtFull only: each of nblk workgroups (kCcLocalGroups,
// fewer on grids with fewer tiles, more where a thread per tile would not cover them) reads the
// kinds of every nblk-th tile (at most one per thread), lists its kCtFull tiles in LDS and labels
// them one after the other. The list's order is that of the LDS atomics;
// each tile is labelled on its own, so the results do not depend on it.
constexpr int64_t kCcLocalGroups = 1024;

inline unsigned cc_local_groups(int64_t ntiles)
{
    const int64_t need = (ntiles + kCtBoxes - 1) / kCtBoxes;
    const int64_t gr = ntiles < kCcLocalGroups ? ntiles : kCcLocalGroups;
    return (unsigned)(gr > need ? gr : need);
}

struct KCcLocal {
    static constexpr int kThreads = kCtBoxes, kWaves = 0;
    struct Args {
        Grid g;
        const uint8_t *label;
        uint8_t phase;
        uint32_t *parent;
        uint32_t *csize;
        uint32_t *psize;
        const uint8_t *ctile;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCcLocal::run(const Args &args_, uint32_t blk, uint32_t nblk)
{
    Grid g = args_.g;
    const uint8_t *label = args_.label;
    uint8_t phase = args_.phase;
    uint32_t *parent = args_.parent;
    uint32_t *csize = args_.csize;
    uint32_t *psize = args_.psize;
    __shared__ uint32_t lp[kCtBoxes];
    __shared__ uint32_t lc[kCtBoxes];
    const int ntx = (g.n[0] + CT - 1) / CT, nty = (g.n[1] + CT - 1) / CT;
    const int l = threadIdx.x;
    const int lx = l % CT, ly = (l / CT) % CT, lz = l / (CT * CT);
    const int64_t ntiles = (int64_t)ntx * nty * ((g.n[2] + CT - 1) / CT);
    __shared__ int list[kCtBoxes];
    __shared__ uint32_t count;
    if (l == 0) count = 0u;
    __syncthreads();
    const int64_t t = blk + (int64_t)l * nblk;
    if (t < ntiles && args_.ctile[t] == kCtFull) list[atomicAdd(&count, 1u)] = (int)t;
    __syncthreads();
    const uint32_t m = count;
    for (uint32_t q = 0; q < m; ++q) {
        const int b = list[q];
        const int x0 = (b % ntx) * CT, y0 = ((b / ntx) % nty) * CT, z0 = (b / (ntx * nty)) * CT;
        const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
        const bool in = gx < g.n[0] && gy < g.n[1] && gz < g.n[2];
        const int64_t c = in ? lin(g, gx, gy, gz) : 0;
        const bool mine = in && label[c] == phase;
        // the previous tile's LDS reads are done (and the counts below are uniform)
        const int nmine = __syncthreads_count(mine), nin = __syncthreads_count(in);
        if (nmine == nin) {
            // every in-grid box has the phase (fewer than `limit`): one box-shaped piece whose
            // smallest member is the tile's first box
            if (in) {
                csize[c] = 0;
                parent[c] = (uint32_t)lin(g, x0, y0, z0);
                psize[c] = (uint32_t)nmine;
            }
            continue;
        }
        lp[l] = mine ? (uint32_t)l : kInvalid;
        lc[l] = 0;
        __syncthreads();
        if (mine) {
            if (lx + 1 < CT && gx + 1 < g.n[0] && lp[l + 1] != kInvalid) lunite(lp, l, l + 1);
            if (ly + 1 < CT && gy + 1 < g.n[1] && lp[l + CT] != kInvalid) lunite(lp, l, l + CT);
            if (lz + 1 < CT && gz + 1 < g.n[2] && lp[l + CT * CT] != kInvalid) lunite(lp, l, l + CT * CT);
        }
        __syncthreads();
        uint32_t r = mine ? lfind(lp, l) : 0u;
        if (mine) atomicAdd(lc + r, 1u);
        __syncthreads();
        if (in) {
            if (mine) {
                csize[c] = 0;
                int rx = r % CT, ry = (r / CT) % CT, rz = r / (CT * CT);
                parent[c] = (uint32_t)lin(g, x0 + rx, y0 + ry, z0 + rz);
                psize[c] = lc[r];
            } else {
                parent[c] = kInvalid;
            }
        }
    }
}

// Joins across tile faces (and the periodic faces of the grid): only boxes on a tile's upper
// faces look at their +x / +y / +z neighbour. Only "fewer than `limit` boxes" matters, and a
// piece that already has `limit` boxes inside its tile is large whatever it joins, so a face
// is joined only when at least one of its two pieces is small; a small piece still ends in
// the same tree as every piece it touches. When a small piece joins a large one, the large
// side's face box is tagged (psize = kTouched) so that the size count below sees the tree as
// large.
constexpr uint32_t kTouched = 0xffffffffu;

struct KCcMerge {
    // one workgroup per component tile, a lane per box of its three upper faces (x, y, z)
    static constexpr int kThreads = 3 * CT * CT, kWaves = 0;
    struct Args {
        Grid g;
        const uint8_t *label;
        uint8_t phase;
        uint32_t *parent;
        uint32_t *psize;
        uint32_t limit;
        const uint8_t *ctile;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCcMerge::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    const uint8_t *label = args_.label;
    const uint8_t phase = args_.phase;
    uint32_t *parent = args_.parent;
    uint32_t *psize = args_.psize;
    const uint32_t limit = args_.limit;
    const uint8_t *ctile = args_.ctile;
    const uint8_t kind = ctile[blk];
    if (kind == kCtNone) return;                    // no box of the phase here
    const int ntx = (g.n[0] + CT - 1) / CT, nty = (g.n[1] + CT - 1) / CT;
    const int b = blk;
    const int x0 = (b % ntx) * CT, y0 = ((b / ntx) % nty) * CT, z0 = (b / (ntx * nty)) * CT;
    // a tile's upper face in an axis is its last in-grid layer (the grid's last layer joins the
    // first one across the periodic face)
    const int nx = min(CT, (int)g.n[0] - x0), ny = min(CT, (int)g.n[1] - y0), nz = min(CT, (int)g.n[2] - z0);
    const int q = threadIdx.x / (CT * CT);
    const int u = threadIdx.x % CT, v = (threadIdx.x / CT) % CT;
    const int lx = q == 0 ? nx - 1 : u, ly = q == 1 ? ny - 1 : (q == 0 ? u : v), lz = q == 2 ? nz - 1 : v;
    if (lx >= nx || ly >= ny || lz >= nz) return;
    const int i = x0 + lx, j = y0 + ly, k = z0 + lz;
    const int64_t c = lin(g, i, j, k);
    if (label[c] != phase) return;
    const int ip = q == 0 ? (i + 1 == g.n[0] ? 0 : i + 1) : i;
    const int jp = q == 1 ? (j + 1 == g.n[1] ? 0 : j + 1) : j;
    const int kp = q == 2 ? (k + 1 == g.n[2] ? 0 : k + 1) : k;
    const int64_t nb = lin(g, ip, jp, kp);
    if (label[nb] != phase) return;
    // A box of a kCtLarge tile belongs to a large piece without union-find entries: a small
    // piece touching it is tagged (psize = kTouched, which the size count reads as "large")
    // instead of joined. Otherwise piece sizes only move to kTouched (>= limit) while this
    // runs, and a face is joined when at least one of its two pieces can still be small (a box
    // on several faces takes each face in its own lane; the outcome does not depend on their
    // timing).
    const bool large_tile = kind != kCtFull;
    const bool nlarge_tile = ctile[ct_tile(g, ip, jp, kp)] != kCtFull;
    if (large_tile && nlarge_tile) return;
    if (large_tile) {
        if (psize[nb] < limit) psize[nb] = kTouched;
        return;
    }
    const bool small = psize[c] < limit;
    if (nlarge_tile) {
        if (small) psize[c] = kTouched;
        return;
    }
    const bool nsmall = psize[nb] < limit;
    if (!small && !nsmall) return;
    unite(parent, (uint32_t)c, (uint32_t)nb);
    if (!small) psize[c] = kTouched;
    if (!nsmall) psize[nb] = kTouched;
}

struct KCcFlatten {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        uint32_t *parent;
        const uint8_t *ctile;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCcFlatten::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    uint32_t *parent = args_.parent;
    if (args_.ctile[blk] != kCtFull) return;
    for (int h = 0; h < kCtPer; ++h) {
        int64_t c;
        if (!ct_box(g, blk, (int)threadIdx.x + h * kBlock, c)) continue;
        if (parent[c] == kInvalid) continue;
        parent[c] = find_root(parent, (uint32_t)c);
    }
}

// Component sizes, counted only until they reach `limit` (only "size < limit" matters). Boxes
// of small pieces count one each; a tagged box of a large piece (which joined a small one)
// lifts its tree to `limit`. Trees made of large pieces only hold no small box and are never
// looked at.
struct KCcSize {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        const uint32_t *parent;
        const uint32_t *psize;
        uint32_t *csize;
        uint32_t limit;
        const uint8_t *ctile;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCcSize::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    const uint32_t *parent = args_.parent;
    const uint32_t *psize = args_.psize;
    uint32_t *csize = args_.csize;
    uint32_t limit = args_.limit;
    if (args_.ctile[blk] != kCtFull) return;
    const unsigned lane = __lane_id();
    for (int h = 0; h < kCtPer; ++h) {
        int64_t c = 0;
        const bool in = ct_box(g, blk, (int)threadIdx.x + h * kBlock, c);
        uint32_t r = in ? parent[c] : kInvalid;
        const uint32_t ps = r != kInvalid ? psize[c] : 0u;
        const bool small = r != kInvalid && ps < limit;
        const bool touched = r != kInvalid && ps == kTouched;
        bool active = small || touched;
        const unsigned long long smallmask = __ballot(small), touchedmask = __ballot(touched);
        unsigned long long pending = __ballot(active);
        while (pending) {
            int leader = __ffsll((long long)pending) - 1;
            uint32_t rl = __shfl(r, leader, 64);
            unsigned long long peers = __ballot(active && r == rl);
            if ((int)lane == leader) {
                if (peers & touchedmask) {
                    atomicMax(csize + rl, limit);
                } else {
                    uint32_t cur = __hip_atomic_load(csize + rl, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
                    if (cur < limit) atomicAdd(csize + rl, (uint32_t)__popcll(peers & smallmask));
                }
            }
            if (peers & (1ull << lane)) active = false;
            pending &= ~peers;
        }
    }
}

// Boxes of small components change phase; boxes of large pieces belong to large components.
struct KCcFlip {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        uint8_t *label;
        uint8_t phase;
        const uint32_t *parent;
        const uint32_t *psize;
        const uint32_t *csize;
        uint32_t limit;
        long long *stats;
        int slot;
        const uint8_t *ctile;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCcFlip::run(const Args &args_, uint32_t blk, uint32_t)
{
    const Grid &g = args_.g;
    uint8_t *label = args_.label;
    uint8_t phase = args_.phase;
    const uint32_t *parent = args_.parent;
    const uint32_t *psize = args_.psize;
    const uint32_t *csize = args_.csize;
    uint32_t limit = args_.limit;
    long long *stats = args_.stats;
    int slot = args_.slot;
    if (args_.ctile[blk] != kCtFull) return;
    unsigned long long nf = 0, nr = 0;
    for (int h = 0; h < kCtPer; ++h) {
        int64_t c = 0;
        bool flip = false, root = false;
        if (ct_box(g, blk, (int)threadIdx.x + h * kBlock, c) && label[c] == phase && psize[c] < limit) {
            uint32_t r = parent[c];
            if (csize[r] < limit) {
                flip = true;
                root = r == (uint32_t)c;
                label[c] = (uint8_t)(1 - phase);
            }
        }
        nf += __popcll(__ballot(flip));
        nr += __popcll(__ballot(root));
    }
    if (__lane_id() == 0 && stats) {
        if (nr) atomicAdd((unsigned long long *)(stats + slot), nr);
        if (nf) atomicAdd((unsigned long long *)(stats + slot + 2), nf);
    }
}

// ---- distance (Godunov relaxation) ----------------------------------------------------
__device__ __forceinline__ void cswap(double &a, double &b, double &ha, double &hb, double &wa, double &wb)
{
    if (b < a) {
        double t = a; a = b; b = t;
        t = ha; ha = hb; hb = t;
        t = wa; wa = wb; wb = t;
    }
}

// Larger root of sum_k ((d - a_k)^+ / h_k)^2 = 1 over the axes whose a_k lie below d; w_k is
// 1 / h_k^2, passed in so that the weights are computed once per tile, not per update.
__device__ double godunov(double a0, double a1, double a2, double h0, double h1, double h2, double w0, double w1,
                          double w2)
{
    cswap(a0, a1, h0, h1, w0, w1);
    cswap(a1, a2, h1, h2, w1, w2);
    cswap(a0, a1, h0, h1, w0, w1);
    if (isinf(a0)) return INFINITY;
    double d = a0 + h0;
    if (d > a1) {
        double sw = w0 + w1;
        double swa = w0 * a0 + w1 * a1;
        double dd = a0 - a1;
        double disc = sw - w0 * w1 * (dd * dd);
        if (disc < 0.0) disc = 0.0;
        d = (swa + sqrt(disc)) / sw;
        if (d > a2) {
            sw = w0 + w1 + w2;
            swa = w0 * a0 + w1 * a1 + w2 * a2;
            double d01 = a0 - a1, d02 = a0 - a2, d12 = a1 - a2;
            disc = sw - (w0 * w1 * (d01 * d01) + w0 * w2 * (d02 * d02) + w1 * w2 * (d12 * d12));
            if (disc < 0.0) disc = 0.0;
            d = (swa + sqrt(disc)) / sw;
        }
    }
    return d;
}

// The same root when every axis has the same edge h (w = 1 / h^2): the a_k are sorted by
// minimum and maximum alone (equal edges and weights need not travel with them), then the
// operations above run in the same order on the same operands, so the result is the same to
// the bit.
__device__ double godunov_uniform(double a0, double a1, double a2, double h, double w)
{
    const double lo = fmin(a0, a1), hi = fmax(a0, a1);
    const double b0 = fmin(lo, a2), mid = fmax(lo, a2);
    const double b1 = fmin(mid, hi), b2 = fmax(mid, hi);
    if (isinf(b0)) return INFINITY;
    double d = b0 + h;
    if (d > b1) {
        double sw = w + w;
        double swa = w * b0 + w * b1;
        double dd = b0 - b1;
        double disc = sw - w * w * (dd * dd);
        if (disc < 0.0) disc = 0.0;
        d = (swa + sqrt(disc)) / sw;
        if (d > b2) {
            sw = w + w + w;
            swa = w * b0 + w * b1 + w * b2;
            double d01 = b0 - b1, d02 = b0 - b2, d12 = b1 - b2;
            disc = sw - (w * w * (d01 * d01) + w * w * (d02 * d02) + w * w * (d12 * d12));
            if (disc < 0.0) disc = 0.0;
            d = (swa + sqrt(disc)) / sw;
        }
    }
    return d;
}

// The same root for unit box edges (h = w = 1), as godunov_uniform computes it: every
// multiplication by w or w^2 there is exact and is left out, and the division by 2 is a
// multiplication by 1/2 (exact), so the result is the same to the bit with fewer operations.
__device__ double godunov_unit(double a0, double a1, double a2)
{
    const double lo = fmin(a0, a1), hi = fmax(a0, a1);
    const double b0 = fmin(lo, a2), mid = fmax(lo, a2);
    const double b1 = fmin(mid, hi), b2 = fmax(mid, hi);
    if (isinf(b0)) return INFINITY;
    double d = b0 + 1.0;
    if (d > b1) {
        const double dd = b0 - b1;
        double disc = 2.0 - dd * dd;
        if (disc < 0.0) disc = 0.0;
        d = ((b0 + b1) + sqrt(disc)) * 0.5;
        if (d > b2) {
            const double d01 = b0 - b1, d02 = b0 - b2, d12 = b1 - b2;
            disc = 3.0 - ((d01 * d01 + d02 * d02) + d12 * d12);
            if (disc < 0.0) disc = 0.0;
            d = (((b0 + b1) + b2) + sqrt(disc)) / 3.0;
        }
    }
    return d;
}

// One global relaxation pass over LDS tiles. Two copies of the distance grid alternate;
// cur[t] says which copy holds tile t's values as of the end of the previous pass. A tile
// marked dirty loads its boxes and a one-box halo (each from the copy current for the tile that
// owns it) and relaxes its liquid boxes to local convergence with the halo held fixed, then
// writes the result into its other copy. Inside the tile the boxes are relaxed in red-black
// order: all boxes of one parity of (x + y + z), then all of the other, each reading only
// boxes of the opposite parity, so the outcome does not depend on thread timing and information
// crosses two boxes per sweep. Every read of a pass sees the previous pass's state, so the
// outcome does not depend on the order in which tiles run either. A tile that lowers a value on
// a face marks the tile across that face dirty for the next pass. Passes repeat until one
// changes nothing.
constexpr int TX = 16, TY = 8, TZ = 8;
constexpr int HX = TX + 2, HY = TY + 2, HZ = TZ + 2;
constexpr int kTileThreads = 256;
constexpr int kLocalMax = 128;
static_assert(TX % 2 == 0 && TX * TY * TZ == 4 * kTileThreads, "two boxes of each parity per thread");

__device__ __forceinline__ int tile_of(const Grid &g, int64_t x, int64_t y, int64_t z)
{
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY;
    return (int)(((z / TZ) * nty + y / TY) * ntx + x / TX);
}

// Initial distances (0 on the boxes labelled `zero`, the vapor for the interface distance,
// infinity elsewhere); the tiles holding another box next to a zero box are the only ones the
// first pass can change, and they start dirty.
struct KDistInit {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        const uint8_t *label;
        double *dist;
        uint32_t *dirty;
        uint8_t zero;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KDistInit::run(const Args &args_, uint32_t blk, uint32_t)
{
    Grid g = args_.g;
    const uint8_t *label = args_.label;
    double *dist = args_.dist;
    uint32_t *dirty = args_.dirty;
    const uint8_t zero = args_.zero;
    int64_t c = (int64_t)blk * blockDim.x + threadIdx.x;
    if (c >= g.G) return;
    const bool z0 = label[c] == zero;
    dist[c] = z0 ? 0.0 : INFINITY;
    if (z0) return;
    int64_t i, j, k;
    coords(g, c, i, j, k);
    const int64_t xm = i == 0 ? g.n[0] - 1 : i - 1, xp = i == g.n[0] - 1 ? 0 : i + 1;
    const int64_t ym = j == 0 ? g.n[1] - 1 : j - 1, yp = j == g.n[1] - 1 ? 0 : j + 1;
    const int64_t zm = k == 0 ? g.n[2] - 1 : k - 1, zp = k == g.n[2] - 1 ? 0 : k + 1;
    // the six neighbours' labels loaded together (no short circuit: one round trip, not six)
    const uint8_t n0 = label[lin(g, xm, j, k)], n1 = label[lin(g, xp, j, k)];
    const uint8_t n2 = label[lin(g, i, ym, k)], n3 = label[lin(g, i, yp, k)];
    const uint8_t n4 = label[lin(g, i, j, zm)], n5 = label[lin(g, i, j, zp)];
    const bool front = (n0 == zero) | (n1 == zero) | (n2 == zero) | (n3 == zero) | (n4 == zero) | (n5 == zero);
    if (front) dirty[tile_of(g, i, j, k)] = 1u;
}

__host__ __device__ inline int64_t distance_tile_count(const Grid &g)
{
    return (int64_t)((g.n[0] + TX - 1) / TX) * ((g.n[1] + TY - 1) / TY) * ((g.n[2] + TZ - 1) / TZ);
}

// Passes from kDistLatePass on run in one workgroup (KDistLate), which loops over them until a
// pass changes nothing: by then the solve has converged on the interfaces measured, so they
// cost one launch instead of one each.
constexpr int kDistLatePass = 12;

// The first kDistFullPasses passes launch one workgroup per tile. Later passes, where few tiles
// are dirty or the solve has converged, launch fewer workgroups: each takes every nblk-th tile
// (at most kDistListMax of them), reads their dirty flags at once and relaxes only the dirty
// ones.
constexpr int kDistFullPasses = 8;
constexpr int kDistListMax = 1024;
constexpr int64_t kDistLateGroups = 256;

inline unsigned distance_groups(int64_t ntiles, int it)
{
    if (it < kDistFullPasses) return (unsigned)ntiles;
    int64_t gr = ntiles < kDistLateGroups ? ntiles : kDistLateGroups;
    const int64_t need = (ntiles + kDistListMax - 1) / kDistListMax;
    return (unsigned)(gr > need ? gr : need);
}

struct KDistTiles {
    static constexpr int kThreads = kTileThreads, kWaves = 0;
    struct Args {
        Grid g;
        const uint8_t *label;
        double *d0;
        double *d1;
        double cap;
        uint32_t *changed;
        uint32_t *dirty;
        uint32_t *cur;
        int it;
        uint8_t zero;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

// One tile of one pass (b uniform over the workgroup).
__device__ __forceinline__ void dist_tile(const KDistTiles::Args &args_, int b, int ntiles);

__device__ void KDistTiles::run(const Args &args_, uint32_t blk, uint32_t nblk)
{
    const int it = args_.it;
    // once a pass has changed nothing, later passes leave every array as it is (the gather
    // takes the copy flags of the last pass that ran)
    if (it > 0 && __hip_atomic_load(args_.changed + it - 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == 0)
        return;
    const int ntiles = (int)distance_tile_count(args_.g);
    if ((int)nblk >= ntiles) {
        dist_tile(args_, (int)blk, ntiles);
        return;
    }
    uint32_t *dflag = args_.dirty + (it & 1) * ntiles;
    const uint32_t *cprev = args_.cur + (it & 1) * ntiles;
    uint32_t *cnext = args_.cur + ((it + 1) & 1) * ntiles;
    __shared__ int list[kDistListMax];
    __shared__ uint32_t count;
    if (threadIdx.x == 0) count = 0u;
    __syncthreads();
    // clean tiles carry their copy flag over; dirty ones are listed
    for (int64_t b = blk + (int64_t)threadIdx.x * nblk; b < ntiles; b += (int64_t)kTileThreads * nblk) {
        if (dflag[b]) list[atomicAdd(&count, 1u)] = (int)b;
        else cnext[b] = cprev[b];
    }
    __syncthreads();
    const uint32_t m = count;
    for (uint32_t q = 0; q < m; ++q) {
        __syncthreads();
        dist_tile(args_, list[q], ntiles);
    }
}

// The passes from it0 to the budget in one workgroup: each pass lists its dirty tiles, 256 at a
// time, and relaxes them one after the other. Every tile still reads the previous pass's state
// (the two copies and their flags), so the result is the one separate launches would give; the
// workgroup's barriers order its own writes before the next pass reads them.
struct KDistLate {
    static constexpr int kThreads = kTileThreads, kWaves = 0;
    struct Args {
        KDistTiles::Args t;
        int it0;
        int max_sweeps;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KDistLate::run(const Args &args_, uint32_t, uint32_t)
{
    KDistTiles::Args a = args_.t;
    const int ntiles = (int)distance_tile_count(a.g);
    __shared__ int list[kTileThreads];
    __shared__ uint32_t count;
    for (int it = args_.it0; it < args_.max_sweeps; ++it) {
        __syncthreads();
        if (it > 0 && a.changed[it - 1] == 0) break;
        a.it = it;
        const uint32_t *dflag = a.dirty + (it & 1) * ntiles;
        const uint32_t *cprev = a.cur + (it & 1) * ntiles;
        uint32_t *cnext = a.cur + ((it + 1) & 1) * ntiles;
        for (int b0 = 0; b0 < ntiles; b0 += kTileThreads) {
            if (threadIdx.x == 0) count = 0u;
            __syncthreads();
            const int b = b0 + (int)threadIdx.x;
            if (b < ntiles) {
                if (dflag[b]) list[atomicAdd(&count, 1u)] = b;
                else cnext[b] = cprev[b];
            }
            __syncthreads();
            const uint32_t m = count;
            for (uint32_t q = 0; q < m; ++q) {
                __syncthreads();
                dist_tile(a, list[q], ntiles);
            }
            __syncthreads();
        }
    }
}

__device__ __forceinline__ void dist_tile(const KDistTiles::Args &args_, int b, int ntiles)
{
    Grid g = args_.g;
    const uint8_t *label = args_.label;
    double *d0 = args_.d0;
    double *d1 = args_.d1;
    double cap = args_.cap;
    uint32_t *changed = args_.changed;
    uint32_t *dirty = args_.dirty;
    uint32_t *cur = args_.cur;
    int it = args_.it;
    const uint8_t zero = args_.zero;
    uint32_t *dflag = dirty + (it & 1) * ntiles, *dnext = dirty + ((it + 1) & 1) * ntiles;
    const uint32_t *cprev = cur + (it & 1) * ntiles;
    uint32_t *cnext = cur + ((it + 1) & 1) * ntiles;
    const uint32_t mycur = cprev[b];
    if (dflag[b] == 0) {
        if (threadIdx.x == 0) { cnext[b] = mycur; dflag[b] = 0u; }
        return;
    }
    __shared__ double t[HZ][HY][HX];
    __shared__ int faces[6];
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY, ntz = (g.n[2] + TZ - 1) / TZ;
    const int bx = b % ntx, by = (b / ntx) % nty, bz = b / (ntx * nty);
    const int x0 = bx * TX, y0 = by * TY, z0 = bz * TZ;
    if (threadIdx.x < 6) faces[threadIdx.x] = 0;
    // which copy is current for this tile and its 26 periodic neighbours (the owners of every
    // halo box)
    __shared__ uint32_t ncur[27];
    if (threadIdx.x < 27) {
        const int dx = threadIdx.x % 3 - 1, dy = (threadIdx.x / 3) % 3 - 1, dz = threadIdx.x / 9 - 1;
        const int nx = (bx + dx + ntx) % ntx, ny = (by + dy + nty) % nty, nz = (bz + dz + ntz) % ntz;
        ncur[threadIdx.x] = cprev[(nz * nty + ny) * ntx + nx];
    }
    __syncthreads();
    // positions one box outside the grid hold the periodic neighbour (the only outside
    // positions a grid box reads); positions further out (partial tiles) hold infinity. The
    // loads of a thread's halo positions and labels are issued together, with no branch around
    // them, so that a tile waits for one round trip to memory instead of one per load.
    constexpr int kHalo = HX * HY * HZ;
    constexpr int kHaloPer = (kHalo + kTileThreads - 1) / kTileThreads;
    constexpr int kHaloBatch = 4;      // loads in flight per thread (registers: 2 per load)
    static_assert(kHaloPer % kHaloBatch == 0, "whole batches");
#pragma unroll 1
    for (int it0 = 0; it0 < kHaloPer; it0 += kHaloBatch) {
        double hv[kHaloBatch];
#pragma unroll
        for (int u = 0; u < kHaloBatch; ++u) {
            const int q = (int)threadIdx.x + (it0 + u) * kTileThreads;
            const int hx = q % HX, hy = (q / HX) % HY, hz = q / (HX * HY);
            const int gx = x0 + hx - 1, gy = y0 + hy - 1, gz = z0 + hz - 1;
            const bool ok = q < kHalo && gx <= g.n[0] && gy <= g.n[1] && gz <= g.n[2];
            const int cx = gx < 0 ? gx + g.n[0] : (gx == g.n[0] ? 0 : gx);
            const int cy = gy < 0 ? gy + g.n[1] : (gy == g.n[1] ? 0 : gy);
            const int cz = gz < 0 ? gz + g.n[2] : (gz == g.n[2] ? 0 : gz);
            // owner tile relative to this one, -1, 0 or +1 per axis after the periodic wrap
            int ox = cx / TX - bx, oy = cy / TY - by, oz = cz / TZ - bz;
            ox = ox > 1 ? ox - ntx : (ox < -1 ? ox + ntx : ox);
            oy = oy > 1 ? oy - nty : (oy < -1 ? oy + nty : oy);
            oz = oz > 1 ? oz - ntz : (oz < -1 ? oz + ntz : oz);
            const int nq = ok ? (oz + 1) * 9 + (oy + 1) * 3 + (ox + 1) : 13;
            const double *src = ncur[nq] ? d1 : d0;
            const double v = src[ok ? lin(g, cx, cy, cz) : 0];
            hv[u] = ok ? v : INFINITY;
        }
#pragma unroll
        for (int u = 0; u < kHaloBatch; ++u) {
            const int q = (int)threadIdx.x + (it0 + u) * kTileThreads;
            if (q < kHalo) t[q / (HX * HY)][(q / HX) % HY][q % HX] = hv[u];
        }
    }
    // this thread's boxes: the m-th (m = 0, 1) box of parity p, counting along x-rows, which
    // hold TX / 2 boxes of each parity
    int bxs[2][2], bys[2][2], bzs[2][2];
    bool liq[2][2];
#pragma unroll
    for (int p = 0; p < 2; ++p)
#pragma unroll
        for (int m = 0; m < 2; ++m) {
            const int kk = threadIdx.x + m * kTileThreads;
            const int row = kk / (TX / 2), pos = kk % (TX / 2);
            const int ly = row % TY, lz = row / TY;
            const int lx = 2 * pos + ((ly + lz + p) & 1);
            bxs[p][m] = lx + 1; bys[p][m] = ly + 1; bzs[p][m] = lz + 1;
            const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
            const bool in = gx < g.n[0] && gy < g.n[1] && gz < g.n[2];
            liq[p][m] = in && label[in ? lin(g, gx, gy, gz) : 0] != zero;
        }
    const double wx = 1.0 / (g.h[0] * g.h[0]), wy = 1.0 / (g.h[1] * g.h[1]), wz = 1.0 / (g.h[2] * g.h[2]);
    const bool uniform = g.h[0] == g.h[1] && g.h[1] == g.h[2];
    const bool unit = uniform && g.h[0] == 1.0;
    __syncthreads();
    // the loaded values of this thread's boxes (the tile's own copy), to detect changes
    double init[2][2];
    for (int p = 0; p < 2; ++p)
        for (int m = 0; m < 2; ++m) init[p][m] = t[bzs[p][m]][bys[p][m]][bxs[p][m]];
    // the upwind neighbour values each box was last updated from (NaN: not yet). An update
    // from the same values gives the same candidate, which cannot lower the box again, so it
    // is skipped; only boxes next to a change redo the quadratic solve.
    double seen[2][2][3];
    for (int p = 0; p < 2; ++p)
        for (int m = 0; m < 2; ++m) seen[p][m][0] = seen[p][m][1] = seen[p][m][2] = NAN;
    bool local_done = false;
    for (int sweep = 0; sweep < kLocalMax; ++sweep) {
        bool ch = false;
        for (int p = 0; p < 2; ++p) {
            for (int m = 0; m < 2; ++m) {
                if (!liq[p][m]) continue;
                const int hx = bxs[p][m], hy = bys[p][m], hz = bzs[p][m];
                const double ax = fmin(t[hz][hy][hx - 1], t[hz][hy][hx + 1]);
                const double ay = fmin(t[hz][hy - 1][hx], t[hz][hy + 1][hx]);
                const double az = fmin(t[hz - 1][hy][hx], t[hz + 1][hy][hx]);
                if (ax == seen[p][m][0] && ay == seen[p][m][1] && az == seen[p][m][2]) continue;
                seen[p][m][0] = ax; seen[p][m][1] = ay; seen[p][m][2] = az;
                if (isinf(ax) && isinf(ay) && isinf(az)) continue;
                const double old = t[hz][hy][hx];
                const double db = unit ? godunov_unit(ax, ay, az)
                                       : uniform ? godunov_uniform(ax, ay, az, g.h[0], wx)
                                                 : godunov(ax, ay, az, g.h[0], g.h[1], g.h[2], wx, wy, wz);
                if (db <= cap && db < old) { t[hz][hy][hx] = db; ch = true; }
            }
            if (p == 0) __syncthreads();
        }
        if (!__syncthreads_or(ch)) { local_done = true; break; }
    }
    // write back into the tile's other copy (only if something changed)
    bool wrote = false;
    for (int p = 0; p < 2; ++p)
        for (int m = 0; m < 2; ++m) {
            const int lx = bxs[p][m] - 1, ly = bys[p][m] - 1, lz = bzs[p][m] - 1;
            const int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
            if (gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) continue;
            if (t[lz + 1][ly + 1][lx + 1] < init[p][m]) {
                wrote = true;
                if (lx == 0) faces[0] = 1;
                if (lx == TX - 1 || gx == g.n[0] - 1) faces[1] = 1;
                if (ly == 0) faces[2] = 1;
                if (ly == TY - 1 || gy == g.n[1] - 1) faces[3] = 1;
                if (lz == 0) faces[4] = 1;
                if (lz == TZ - 1 || gz == g.n[2] - 1) faces[5] = 1;
            }
        }
    const bool tile_wrote = __syncthreads_or(wrote);
    if (tile_wrote) {
        double *dst = mycur ? d0 : d1;
        for (int q = threadIdx.x; q < TX * TY * TZ; q += kTileThreads) {
            int lx = q % TX, ly = (q / TX) % TY, lz = q / (TX * TY);
            int gx = x0 + lx, gy = y0 + ly, gz = z0 + lz;
            if (gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) continue;
            dst[lin(g, gx, gy, gz)] = t[lz + 1][ly + 1][lx + 1];
        }
    }
    if (threadIdx.x == 0) {
        cnext[b] = tile_wrote ? 1u - mycur : mycur;
        dflag[b] = 0u;
        if (tile_wrote) {
            changed[it] = 1u;
            const int nbx[2] = {bx == 0 ? ntx - 1 : bx - 1, bx == ntx - 1 ? 0 : bx + 1};
            const int nby[2] = {by == 0 ? nty - 1 : by - 1, by == nty - 1 ? 0 : by + 1};
            const int nbz[2] = {bz == 0 ? ntz - 1 : bz - 1, bz == ntz - 1 ? 0 : bz + 1};
            for (int f = 0; f < 2; ++f) {
                if (faces[f]) dnext[(bz * nty + by) * ntx + nbx[f]] = 1u;
                if (faces[2 + f]) dnext[(bz * nty + nby[f]) * ntx + bx] = 1u;
                if (faces[4 + f]) dnext[(nbz[f] * nty + by) * ntx + bx] = 1u;
            }
            // a tile stopped by the sweep limit runs again
            if (!local_done) dnext[b] = 1u;
        }
    }
}

// Final values into d0: boxes whose tile ended with the second copy current are copied. The
// copy flags are those written by the last pass that ran: the first pass that changed nothing
// (later passes exit at once), or the last pass of the budget.
struct KDistGather {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        double *d0;
        const double *d1;
        const uint32_t *cur;        // [2][tiles] copy flags of even / odd passes
        const uint32_t *changed;    // [max_sweeps] per-pass change flags
        int max_sweeps;
        int ntiles;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KDistGather::run(const Args &args_, uint32_t blk, uint32_t)
{
    Grid g = args_.g;
    double *d0 = args_.d0;
    const double *d1 = args_.d1;
    int last = args_.max_sweeps - 1;
    for (int q = 0; q < args_.max_sweeps; ++q)
        if (args_.changed[q] == 0) { last = q; break; }
    const uint32_t *cur_final = args_.cur + ((last + 1) & 1) * args_.ntiles;
    // one workgroup per tile: only tiles that ended in the second copy move anything
    if (!cur_final[blk]) return;
    const int ntx = (g.n[0] + TX - 1) / TX, nty = (g.n[1] + TY - 1) / TY;
    const int x0 = (int)(blk % ntx) * TX, y0 = (int)((blk / ntx) % nty) * TY, z0 = (int)(blk / (ntx * nty)) * TZ;
    for (int q = threadIdx.x; q < TX * TY * TZ; q += kBlock) {
        const int gx = x0 + q % TX, gy = y0 + (q / TX) % TY, gz = z0 + q / (TX * TY);
        if (gx >= g.n[0] || gy >= g.n[1] || gz >= g.n[2]) continue;
        const int64_t c = lin(g, gx, gy, gz);
        d0[c] = d1[c];
    }
}

// Sweep count and the not-converged flag; then the per-pass change flags, tile dirty flags and
// tile copy flags go back to zero, as the next solve expects them.
struct KDistFinish {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        uint32_t *changed;
        int max_sweeps;
        long long *sweeps;
        uint32_t *flags;
        uint32_t *dirty;   // [2][tiles]
        uint32_t *cur;     // [2][tiles]
        int64_t ntiles;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KDistFinish::run(const Args &args_, uint32_t blk, uint32_t nblk)
{
    uint32_t *changed = args_.changed;
    const int max_sweeps = args_.max_sweeps;
    if (blk == 0) {
        if (threadIdx.x == 0) {
            int used = max_sweeps;
            for (int s = 0; s < max_sweeps; ++s)
                if (changed[s] == 0) { used = s + 1; break; }
            if (args_.sweeps) *args_.sweeps = used;
            if (changed[max_sweeps - 1] != 0) atomicOr(args_.flags, kFlagNotConverged);
        }
        __syncthreads();
        for (int q = threadIdx.x; q <= max_sweeps; q += kThreads) changed[q] = 0u;
    }
    for (int64_t q = (int64_t)blk * kThreads + threadIdx.x; q < 2 * args_.ntiles; q += (int64_t)nblk * kThreads) {
        args_.dirty[q] = 0u;
        args_.cur[q] = 0u;
    }
}

struct KCapCopy {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        const double *dist;
        double cap;
        double *out;
        int64_t G;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCapCopy::run(const Args &args_, uint32_t blk, uint32_t)
{
    const double *dist = args_.dist;
    double cap = args_.cap;
    double *out = args_.out;
    int64_t G = args_.G;
    int64_t c = (int64_t)blk * blockDim.x + threadIdx.x;
    if (c < G) out[c] = fmin(dist[c], cap);
}

// ---- per-particle distance and cutoff -------------------------------------------------
__device__ __forceinline__ double lerp(double a, double b, double t) { return a + t * (b - a); }

struct KCutoffs {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        PSet s;
        int64_t n;
        const double *dist;
        const double *dist_v;   // NULL unless vapor particles get dynamic cutoffs too
        double cap;
        double rc_min;
        double rc_max;
        double alpha;
        double a;
        double b;
        int linear;
    };
    static __device__ void run(const Args &args_, uint32_t blk, uint32_t nblk);
};

__device__ void KCutoffs::run(const Args &args_, uint32_t blk, uint32_t)
{
    Grid g = args_.g;
    PSet s = args_.s;
    int64_t n = args_.n;
    const double *dist = args_.dist;
    double cap = args_.cap;
    double rc_min = args_.rc_min;
    double rc_max = args_.rc_max;
    double alpha = args_.alpha;
    double a = args_.a;
    double b = args_.b;
    int linear = args_.linear;
    int64_t p = (int64_t)blk * blockDim.x + threadIdx.x;
    if (p >= n) return;
    double4 q = s.pos[p];
    double x[3] = {q.x, q.y, q.z};
    int64_t i0[3], i1[3];
    double t[3];
    for (int k = 0; k < 3; ++k) {
        double u = x[k] / g.h[k] - 0.5;
        if (!isfinite(u)) u = 0.0;                 // keeps the gathers inside the grid
        double f = floor(u);
        t[k] = u - f;
        int64_t fi = (int64_t)f % g.n[k];
        if (fi < 0) fi += g.n[k];
        i0[k] = fi;
        i1[k] = fi + 1 == g.n[k] ? 0 : fi + 1;
    }
    auto interp = [&](const double *D) {
#define DV(ii, jj, kk) fmin(D[lin(g, ii, jj, kk)], cap)
        double c00 = lerp(DV(i0[0], i0[1], i0[2]), DV(i1[0], i0[1], i0[2]), t[0]);
        double c10 = lerp(DV(i0[0], i1[1], i0[2]), DV(i1[0], i1[1], i0[2]), t[0]);
        double c01 = lerp(DV(i0[0], i0[1], i1[2]), DV(i1[0], i0[1], i1[2]), t[0]);
        double c11 = lerp(DV(i0[0], i1[1], i1[2]), DV(i1[0], i1[1], i1[2]), t[0]);
#undef DV
        double c0 = lerp(c00, c10, t[1]);
        double c1 = lerp(c01, c11, t[1]);
        return lerp(c0, c1, t[2]);
    };
    double d = interp(dist);
    // vapor particles too: the larger of the two depths mirrors Eq. 7 about the interface
    if (args_.dist_v) d = fmax(d, interp(args_.dist_v));
    double rc;
    if (rc_min == rc_max || d <= 0.0) rc = rc_max;
    else if (d >= rc_max) rc = rc_min;
    else if (linear) rc = rc_max + (rc_min - rc_max) * (d / rc_max);
    else rc = a * exp2(alpha * (rc_max - d)) + b;
    q.w = rc;
    s.pos[p] = q;
}

}  // namespace

void launch_count_from_ranges(const Grid &g, const uint32_t *cell_start, uint32_t *out, hipStream_t st)
{
    emit<KCountFromRanges>({g, cell_start, out}, grid1(g.G), st);
}

// `passes` rounds of x, y, z [1,2,1] passes over the box counts taken from the cell ranges
// when cell_start is given (else over `in`); the result always ends in `out`.
void launch_smooth(const Grid &g, int passes, const uint32_t *cell_start, const uint32_t *in,
                   uint32_t *out, uint32_t *tmp, hipStream_t st)
{
    if (passes == 0) {
        if (cell_start) launch_count_from_ranges(g, cell_start, out, st);
        else if (in != out) launch_copy_bytes(out, in, sizeof(uint32_t) * (size_t)g.G, st);
        return;
    }
    const int total = passes;
    const unsigned blocks = (unsigned)(((g.n[0] + SX - 1) / SX) * ((g.n[1] + SY - 1) / SY) * ((g.n[2] + SZ - 1) / SZ));
    const uint32_t *src = in;
    if (cell_start) {
        // the box counts (Eq. 9) as an image first, in the buffer the first pass does not write
        uint32_t *counts = (total % 2 == 1) ? tmp : out;
        launch_count_from_ranges(g, cell_start, counts, st);
        src = counts;
    }
    for (int s = 0; s < total; ++s) {
        uint32_t *dst = ((total - 1 - s) % 2 == 0) ? out : tmp;
        emit<KSmooth3>({g, src, dst}, blocks, st);
        src = dst;
    }
}

void launch_two_means(const Grid &g, const uint32_t *img, GridWork w, long long *stats_out,
                      bool hist_zero, hipStream_t st)
{
    if (!hist_zero) launch_fill_u32(w.hist, 0u, kHistBins, st);
    unsigned nb = (unsigned)std::min<int64_t>((g.G + kBlock - 1) / kBlock, 512);
    emit<KHist>({img, g.G, w.hist, w.flags, ((uintptr_t)img & 15u) == 0}, nb, st);
    emit<KTwoMeans>({w.hist, w.km, stats_out}, 1, st);
}

void launch_segment(const Grid &g, const uint32_t *img, const double *km, int32_t min_component,
                    const MsParams &ms, GridWork w, hipStream_t st)
{
    emit<KThreshold>({img, km, g.G, w.raw, w.label}, grid1(g.G), st);
    if (ms.nu > 0.0) launch_mumford_shah(g, img, km, ms, w.raw, w.label, w.ms, st);
    if (min_component <= 1) return;                 // no component can be smaller
    for (int pass = 0; pass < 2; ++pass) {
        uint8_t phase = pass == 0 ? 1 : 0;
        unsigned nct = (unsigned)(((g.n[0] + CT - 1) / CT) * ((g.n[1] + CT - 1) / CT) * ((g.n[2] + CT - 1) / CT));
        const uint32_t limit = (uint32_t)min_component;
        emit<KCcClassify>({g, w.label, phase, w.ctile, limit}, nct, st);
        emit<KCcLocal>({g, w.label, phase, w.parent, w.csize, w.gtmp, w.ctile}, cc_local_groups(nct), st);
        emit<KCcMerge>({g, w.label, phase, w.parent, w.gtmp, limit, w.ctile}, nct, st);
        emit<KCcFlatten>({g, w.parent, w.ctile}, nct, st);
        emit<KCcSize>({g, w.parent, (const uint32_t *)w.gtmp, w.csize, limit, w.ctile}, nct, st);
        emit<KCcFlip>({g, w.label, phase, w.parent, (const uint32_t *)w.gtmp, w.csize, limit, w.stats,
                       1 + pass, w.ctile}, nct, st);
    }
}

int64_t component_tiles(const Grid &g)
{
    return (int64_t)((g.n[0] + CT - 1) / CT) * ((g.n[1] + CT - 1) / CT) * ((g.n[2] + CT - 1) / CT);
}

int64_t distance_tiles(const Grid &g) { return distance_tile_count(g); }

// Global passes needed: the band depth in tiles plus slack; reaching the bound is reported.
int max_distance_sweeps(const Grid &g, double cap)
{
    double hmin = std::min(g.h[0], std::min(g.h[1], g.h[2]));
    int depth = (int)std::ceil(cap / hmin);
    return depth / std::min(TX, std::min(TY, TZ)) + 24;
}

void launch_distance(const Grid &g, double cap, const uint8_t *label, uint8_t zero, double *dist,
                     GridWork w, long long *sweeps, bool flags_zero, hipStream_t st)
{
    int ms = max_distance_sweeps(g, cap);
    const unsigned ntiles = (unsigned)distance_tiles(g);
    if (!flags_zero) {
        launch_fill_u32(w.changed, 0u, ms + 1, st);
        launch_fill_u32(w.tdirty, 0u, 2 * (int64_t)ntiles, st);
        launch_fill_u32(w.tcur, 0u, 2 * (int64_t)ntiles, st);
    }
    emit<KDistInit>({g, label, dist, w.tdirty, zero}, grid1(g.G), st);
    const int it0 = ms < kDistLatePass ? ms : kDistLatePass;
    for (int it = 0; it < it0; ++it)
        emit<KDistTiles>({g, label, dist, w.dist2, cap, w.changed, w.tdirty, w.tcur, it, zero},
                         distance_groups(ntiles, it), st);
    if (it0 < ms)
        emit<KDistLate>({{g, label, dist, w.dist2, cap, w.changed, w.tdirty, w.tcur, it0, zero}, it0, ms}, 1, st);
    emit<KDistGather>({g, dist, (const double *)w.dist2, w.tcur, w.changed, ms, (int)ntiles}, ntiles, st);
    const unsigned fb = grid1(2 * (int64_t)ntiles);
    emit<KDistFinish>({w.changed, ms, sweeps, w.flags, w.tdirty, w.tcur, (int64_t)ntiles}, fb < 256u ? fb : 256u, st);
}

void launch_distance_flags_zero(const Grid &g, double cap, GridWork w, hipStream_t st)
{
    launch_fill_u32(w.changed, 0u, max_distance_sweeps(g, cap) + 1, st);
    const int64_t ntiles = distance_tiles(g);
    launch_fill_u32(w.tdirty, 0u, 2 * ntiles, st);
    launch_fill_u32(w.tcur, 0u, 2 * ntiles, st);
}

void launch_cap_copy(const double *dist, double cap, double *out, int64_t G, hipStream_t st)
{
    emit<KCapCopy>({dist, cap, out, G}, grid1(G), st);
}

void launch_cutoffs(const Grid &g, PSet s, int64_t n, const double *dist, const double *dist_v, double cap,
                    double rc_min, double rc_max, double alpha, double a, double b, int linear, hipStream_t st)
{
    emit<KCutoffs>({g, s, n, dist, dist_v, cap, rc_min, rc_max, alpha, a, b, linear}, grid1(n), st);
}

}  // namespace dcm
