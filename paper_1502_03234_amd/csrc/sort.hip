// sort.hip -- binning of particles into boxes by sort-and-segment (Section 4, Eq. 9-10).
//
// Each particle gets the linear index of the box containing it (x fastest). The particles
// are then sorted by that key with a stable LSD radix sort whose per-tile ranks come from
// wavefront ballots (no atomics anywhere), the first slot of every box is found where the
// sorted key changes, and slots inside a box are ordered by particle id so that the
// internal order -- and with it every summation order -- is a function of the state alone.
// The box counts b_ijk of Eq. 9 are differences of consecutive box starts.
#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

constexpr int kRadixBits = 8;
constexpr int kDigits = 1 << kRadixBits;
constexpr int kItems = 8;                          // keys per thread per tile
constexpr int kBlockWaves = kBlock / 64;
constexpr int kTile = kBlock * kItems;             // 2048 keys per tile

__device__ __forceinline__ double wrap1(double x, double L)
{
    double t = x - L * floor(x / L);
    if (t < 0.0) t += L;
    if (t >= L) t = 0.0;
    return t;
}

struct KWrapKey {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { Grid g; PSet s; int64_t n; uint32_t *key, *val; };
    static __device__ void run(const Args &args, uint32_t blk, uint32_t);
};

__device__ void KWrapKey::run(const Args &args, uint32_t blk, uint32_t)
{
    const Grid &g = args.g;
    const PSet &s = args.s;
    int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    if (i >= args.n) return;
    double4 p = s.pos[i];
    p.x = wrap1(p.x, g.L[0]);
    p.y = wrap1(p.y, g.L[1]);
    p.z = wrap1(p.z, g.L[2]);
    s.pos[i] = p;
    args.key[i] = pos_key(g, p.x, p.y, p.z);
    args.val[i] = (uint32_t)i;
}

// Box counts of Eq. 9 from the current positions (neighbour-list mode, where particles keep
// their storage order between list builds): count[(c N_y + b) N_x + a] += 1, integer atomics,
// so the counts do not depend on the order of the additions.
struct KCountBoxes {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { Grid g; const double4 *pos; int64_t n; uint32_t *count; };
    static __device__ void run(const Args &args, uint32_t blk, uint32_t)
    {
        const Grid &g = args.g;
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        if (i >= args.n) return;
        const double4 p = args.pos[i];
        const int32_t a = box_index(p.x, g.h[0], g.n[0]);
        const int32_t b = box_index(p.y, g.h[1], g.n[1]);
        const int32_t c = box_index(p.z, g.h[2], g.n[2]);
        atomicAdd(args.count + ((int64_t)c * g.n[1] + b) * g.n[0] + a, 1u);
    }
};

// Validity of the neighbour lists: the largest squared displacement since the build (minimum
// image) and the largest growth of a cutoff, as the bit patterns of non-negative doubles
// (ordered like the values) in out[0] and out[1].
struct KListCheck {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { Grid g; const double4 *pos; const double4 *pos_build; int64_t n; unsigned long long *out; };
    static __device__ void run(const Args &args, uint32_t blk, uint32_t)
    {
        const Grid &g = args.g;
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        double d2 = 0.0, grow = 0.0;
        if (i < args.n) {
            const double4 p = args.pos[i], b = args.pos_build[i];
            double dx = p.x - b.x, dy = p.y - b.y, dz = p.z - b.z;
            dx -= g.L[0] * rint(dx / g.L[0]);
            dy -= g.L[1] * rint(dy / g.L[1]);
            dz -= g.L[2] * rint(dz / g.L[2]);
            d2 = dx * dx + dy * dy + dz * dz;
            grow = fmax(p.w - b.w, 0.0);
            if (!(d2 >= 0.0) || !(p.w == p.w)) d2 = INFINITY;   // a non-finite state rebuilds
        }
        for (int off = 32; off > 0; off >>= 1) {
            d2 = fmax(d2, __shfl_xor(d2, off, 64));
            grow = fmax(grow, __shfl_xor(grow, off, 64));
        }
        if ((threadIdx.x & 63) == 0) {
            atomicMax(args.out, (unsigned long long)__double_as_longlong(d2));
            atomicMax(args.out + 1, (unsigned long long)__double_as_longlong(grow));
        }
    }
};

struct KInitIds {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { PSet s; int64_t n; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        if (i < a.n) a.s.id[i] = (uint32_t)i;
    }
};

__device__ __forceinline__ unsigned lane_id() { return __lane_id(); }

// Lanes of the current wave (among `valid` ones) whose digit equals this lane's.
__device__ __forceinline__ unsigned long long peer_mask(uint32_t digit, bool valid)
{
    unsigned long long peers = __ballot(valid);
#pragma unroll
    for (int b = 0; b < kRadixBits; ++b) {
        bool bit = (digit >> b) & 1u;
        unsigned long long bal = __ballot(bit);
        peers &= bit ? bal : ~bal;
    }
    return peers;
}

// Per-tile digit counts: tile_counts[d * ntiles + t].
struct KRadixCount {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { const uint32_t *key; int64_t n; int shift; uint32_t *tile_counts; int64_t ntiles; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KRadixCount::run(const Args &a, uint32_t blk, uint32_t)
{
    const uint32_t *key = a.key;
    const int64_t n = a.n;
    const int shift = a.shift;
    __shared__ uint32_t whist[kBlockWaves][kDigits];
    const int tid = threadIdx.x, w = tid >> 6;
    const unsigned lane = lane_id();
    for (int d = tid; d < kBlockWaves * kDigits; d += kBlock) (&whist[0][0])[d] = 0;
    __syncthreads();
    const int64_t base = (int64_t)blk * kTile + (int64_t)w * 64 * kItems;
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + r * 64 + lane;
        bool valid = i < n;
        uint32_t digit = valid ? (key[i] >> shift) & (kDigits - 1) : 0u;
        unsigned long long peers = peer_mask(digit, valid);
        unsigned long long lower = peers & ((1ull << lane) - 1ull);
        if (valid && lower == 0ull) whist[w][digit] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    for (int d = tid; d < kDigits; d += kBlock) {
        uint32_t c = 0;
        for (int q = 0; q < kBlockWaves; ++q) c += whist[q][d];
        a.tile_counts[(int64_t)d * a.ntiles + blk] = c;
    }
}

// Exclusive scan of 256 values held one per thread (blockDim == 256); returns the total.
__device__ uint32_t block_exclusive_scan(uint32_t v, uint32_t *out_excl, uint32_t *lds /*[kBlockWaves]*/)
{
    const int tid = threadIdx.x, w = tid >> 6;
    const unsigned lane = lane_id();
    uint32_t incl = v;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        uint32_t t = __shfl_up(incl, off, 64);
        if (lane >= (unsigned)off) incl += t;
    }
    if (lane == 63) lds[w] = incl;
    __syncthreads();
    uint32_t wbase = 0, total = 0;
    for (int q = 0; q < kBlockWaves; ++q) {
        if (q < w) wbase += lds[q];
        total += lds[q];
    }
    *out_excl = wbase + incl - v;
    __syncthreads();
    return total;
}

// One block per digit: exclusive scan of its per-tile counts (in place) and the digit total.
struct KDigitScan {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { uint32_t *tile_counts; int64_t ntiles; uint32_t *digit_total; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KDigitScan::run(const Args &a, uint32_t blk, uint32_t)
{
    __shared__ uint32_t lds[kBlockWaves];
    const int64_t ntiles = a.ntiles;
    uint32_t *row = a.tile_counts + (int64_t)blk * ntiles;
    uint32_t carry = 0;
    for (int64_t start = 0; start < ntiles; start += kBlock * 4) {
        uint32_t v[4], s = 0;
        for (int q = 0; q < 4; ++q) {
            int64_t t = start + (int64_t)threadIdx.x * 4 + q;
            v[q] = t < ntiles ? row[t] : 0u;
            s += v[q];
        }
        uint32_t excl;
        uint32_t total = block_exclusive_scan(s, &excl, lds);
        uint32_t run = carry + excl;
        for (int q = 0; q < 4; ++q) {
            int64_t t = start + (int64_t)threadIdx.x * 4 + q;
            if (t < ntiles) row[t] = run;
            run += v[q];
        }
        carry += total;
    }
    if (threadIdx.x == 0) a.digit_total[blk] = carry;
}

// Stable scatter of one radix pass. The tile's keys are first placed in LDS in tile-local digit
// order, then written out in that order, so consecutive threads write consecutive slots of a
// digit's run in the output.
struct KRadixScatter {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        const uint32_t *key, *val;
        uint32_t *key_out, *val_out;
        int64_t n;
        int shift;
        const uint32_t *tile_prefix;
        int64_t ntiles;
        const uint32_t *digit_total;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KRadixScatter::run(const Args &a, uint32_t blk, uint32_t)
{
    const uint32_t *key = a.key, *val = a.val;
    uint32_t *key_out = a.key_out, *val_out = a.val_out;
    const int64_t n = a.n;
    const int shift = a.shift;
    const uint32_t *tile_prefix = a.tile_prefix, *digit_total = a.digit_total;
    const int64_t ntiles = a.ntiles;
    __shared__ uint32_t whist[kBlockWaves][kDigits];
    __shared__ uint32_t gbase[kDigits];
    __shared__ uint32_t tbase[kDigits];
    __shared__ uint32_t lds[kBlockWaves];
    __shared__ uint32_t sk[kTile], sv[kTile];
    const int tid = threadIdx.x, w = tid >> 6;
    const unsigned lane = lane_id();
    for (int d = tid; d < kBlockWaves * kDigits; d += kBlock) (&whist[0][0])[d] = 0;
    __syncthreads();
    const int64_t tile0 = (int64_t)blk * kTile;
    const int64_t base = tile0 + (int64_t)w * 64 * kItems;
    uint32_t k[kItems], v[kItems], dg[kItems], rk[kItems];
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + r * 64 + lane;
        bool valid = i < n;
        k[r] = valid ? key[i] : 0u;
        v[r] = valid ? val[i] : 0u;
        uint32_t digit = (k[r] >> shift) & (kDigits - 1);
        dg[r] = digit;
        unsigned long long peers = peer_mask(digit, valid);
        unsigned long long lower = peers & ((1ull << lane) - 1ull);
        rk[r] = whist[w][digit] + (uint32_t)__popcll(lower);
        if (valid && lower == 0ull) whist[w][digit] += (uint32_t)__popcll(peers);
    }
    __syncthreads();
    {
        // global digit base = exclusive scan over digit totals + this tile's prefix for the
        // digit; tile-local digit base = exclusive scan over the tile's digit counts; per-wave
        // bases = exclusive scan over the waves of the tile
        uint32_t excl;
        block_exclusive_scan(digit_total[tid], &excl, lds);
        uint32_t acc = 0;
        for (int q = 0; q < kBlockWaves; ++q) {
            uint32_t c = whist[q][tid];
            whist[q][tid] = acc;
            acc += c;
        }
        uint32_t texcl;
        block_exclusive_scan(acc, &texcl, lds);
        tbase[tid] = texcl;
        gbase[tid] = excl + tile_prefix[(int64_t)tid * ntiles + blk];
    }
    __syncthreads();
#pragma unroll
    for (int r = 0; r < kItems; ++r) {
        int64_t i = base + r * 64 + lane;
        if (i < n) {
            const uint32_t p = tbase[dg[r]] + whist[w][dg[r]] + rk[r];
            sk[p] = k[r];
            sv[p] = v[r];
        }
    }
    __syncthreads();
    const int64_t left = n - tile0;
    const int cnt = left < kTile ? (int)left : kTile;
    for (int q = tid; q < cnt; q += kBlock) {
        const uint32_t kk = sk[q];
        const uint32_t d = (kk >> shift) & (kDigits - 1);
        const uint32_t dst = gbase[d] + ((uint32_t)q - tbase[d]);
        key_out[dst] = kk;
        val_out[dst] = sv[q];
    }
}

// Box starts from sorted keys, cell_start[c] = number of keys below c, in two steps. First the
// start of every run of kRangeBoxes keys: the slot where the key changes from a to b starts
// every run whose first key lies in (a, b] (runs before the first key start at 0, after the
// last at n). Then one workgroup per run stages the run's keys in LDS and every box of the run
// finds its start by binary search, so the box starts are written in order.
constexpr int kRangeBoxes = 1024;                   // boxes per run (4 per thread)
constexpr int kRangeKeys = 4096;                    // keys a run can stage in LDS

struct KRunStarts {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { const uint32_t *key; int64_t n, nruns; uint32_t *run_start; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        if (i > a.n) return;
        int64_t lo = (i == 0) ? 0 : (int64_t)(a.key[i - 1] / kRangeBoxes) + 1;
        int64_t hi = (i == a.n) ? a.nruns : (int64_t)(a.key[i] / kRangeBoxes);
        for (int64_t r = lo; r <= hi; ++r) a.run_start[r] = (uint32_t)i;
    }
};

struct KCellRanges {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { const uint32_t *key; int64_t G; const uint32_t *run_start; uint32_t *cell_start; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KCellRanges::run(const Args &args, uint32_t blk, uint32_t)
{
    const uint32_t *key = args.key;
    const int64_t G = args.G;
    uint32_t *cell_start = args.cell_start;
    __shared__ uint32_t sk[kRangeKeys];
    __shared__ uint32_t first[kRangeBoxes];
    __shared__ uint32_t wmin[kBlock / 64];
    constexpr int kPer = kRangeBoxes / kBlock;
    const int64_t c0 = (int64_t)blk * kRangeBoxes;
    const uint32_t lo = args.run_start[blk], hi = args.run_start[blk + 1];
    const uint32_t m = hi - lo;
    if (m > (uint32_t)kRangeKeys) {
        // too many keys to stage: every box finds its start by binary search in global memory
        for (int r = 0; r < kPer; ++r) {
            const int64_t c = c0 + r * kBlock + threadIdx.x;
            if (c > G) break;
            uint32_t a = 0, b = m;
            while (a < b) {
                const uint32_t mid = (a + b) >> 1;
                if ((int64_t)key[lo + mid] < c) a = mid + 1;
                else b = mid;
            }
            cell_start[c] = lo + a;
        }
        return;
    }
    // every key of this run lies in [c0, c0 + kRangeBoxes): the first slot of each key is its
    // box's start; an empty box starts where the next non-empty box of the run does, or at hi
    for (int q = threadIdx.x; q < kRangeBoxes; q += kBlock) first[q] = hi;
    for (uint32_t q = threadIdx.x; q < m; q += kBlock) sk[q] = key[lo + q];
    __syncthreads();
    for (uint32_t q = threadIdx.x; q < m; q += kBlock)
        if (q == 0 || sk[q - 1] != sk[q]) first[sk[q] - (uint32_t)c0] = lo + q;
    __syncthreads();
    // suffix minimum over the boxes: kPer consecutive boxes per thread, then over the threads
    uint32_t v[kPer];
    uint32_t run = 0xffffffffu;
#pragma unroll
    for (int r = kPer - 1; r >= 0; --r) {
        run = min(run, first[threadIdx.x * kPer + r]);
        v[r] = run;
    }
    // inclusive suffix minimum of the per-thread minima within the wave (lanes above)
    const unsigned lane = lane_id();
    uint32_t suf = run;
#pragma unroll
    for (int off = 1; off < 64; off <<= 1) {
        const uint32_t t = __shfl_down(suf, off, 64);
        if (lane + off < 64u) suf = min(suf, t);
    }
    const int w = threadIdx.x >> 6;
    if (lane == 0) wmin[w] = suf;
    __syncthreads();
    // minimum over the later waves and over the later lanes of this wave
    uint32_t after = 0xffffffffu;
    for (int q = w + 1; q < kBlock / 64; ++q) after = min(after, wmin[q]);
    const uint32_t later_lanes = __shfl_down(suf, 1, 64);
    if (lane < 63u) after = min(after, later_lanes);
#pragma unroll
    for (int r = 0; r < kPer; ++r) {
        const int64_t c = c0 + threadIdx.x * kPer + r;
        if (c <= G) cell_start[c] = min(v[r], after);
    }
}

// Inside each storage cell, order slots by particle id (insertion sort; cells hold a few
// particles). One thread per sorted slot: the first slot of a run of equal keys sorts the run.
struct KCellFixup {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { const uint32_t *key; int64_t n; uint32_t *val; const uint32_t *id; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KCellFixup::run(const Args &a, uint32_t blk, uint32_t)
{
    const uint32_t *key = a.key, *id = a.id;
    uint32_t *val = a.val;
    const int64_t s = (int64_t)blk * kThreads + threadIdx.x;
    if (s + 1 >= a.n) return;
    const uint32_t k = key[s];
    if ((s > 0 && key[s - 1] == k) || key[s + 1] != k) return;
    int64_t e = s + 2;
    while (e < a.n && key[e] == k) ++e;
    for (int64_t q = s + 1; q < e; ++q) {
        uint32_t vq = val[q];
        uint32_t iq = id[vq];
        int64_t j = q;
        while (j > s) {
            uint32_t vp = val[j - 1];
            if (id[vp] <= iq) break;
            val[j] = vp;
            --j;
        }
        val[j] = vq;
    }
}

struct KGather {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { PSet from, to; const uint32_t *perm; int64_t n; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KGather::run(const Args &a, uint32_t blk, uint32_t)
{
    const PSet &from = a.from, &to = a.to;
    const uint32_t *perm = a.perm;
    int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    if (i >= a.n) return;
    uint32_t o = perm[i];
    to.pos[i] = from.pos[o];
    to.vx[i] = from.vx[o];
    to.vy[i] = from.vy[o];
    to.vz[i] = from.vz[o];
    to.id[i] = from.id[o];
}

inline unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

}  // namespace

size_t sort_scratch_bytes(int64_t n, int64_t G)
{
    int64_t ntiles = (n + kTile - 1) / kTile;
    int64_t nruns = G / kRangeBoxes + 1;              // runs covering boxes 0..G
    return sizeof(uint32_t) * ((size_t)kDigits * (size_t)ntiles + kDigits + (size_t)nruns + 1);
}

void launch_wrap_key(const Grid &g, PSet s, int64_t n, uint32_t *key, uint32_t *val, hipStream_t st)
{
    emit<KWrapKey>({g, s, n, key, val}, grid1(n), st);
}

void launch_count_boxes(const Grid &g, const double4 *pos, int64_t n, uint32_t *count, hipStream_t st)
{
    launch_fill_u32(count, 0u, g.G, st);
    emit<KCountBoxes>({g, pos, n, count}, grid1(n), st);
}

void launch_list_check(const Grid &g, const double4 *pos, const double4 *pos_build, int64_t n,
                       unsigned long long *out, hipStream_t st)
{
    launch_fill_u32((uint32_t *)out, 0u, 4, st);
    emit<KListCheck>({g, pos, pos_build, n, out}, grid1(n), st);
}

void launch_init_ids(PSet s, int64_t n, hipStream_t st)
{
    emit<KInitIds>({s, n}, grid1(n), st);
}

// Sorts (key, val) by key over the low `bits` bits. The result ends in (key, val): an odd
// number of passes finishes with a copy back from the alternate buffers.
bool launch_radix_sort(uint32_t *key, uint32_t *val, uint32_t *key_alt, uint32_t *val_alt,
                       void *scratch, int64_t n, int bits, hipStream_t st)
{
    int64_t ntiles = (n + kTile - 1) / kTile;
    uint32_t *tile_counts = (uint32_t *)scratch;
    uint32_t *digit_total = tile_counts + (size_t)kDigits * ntiles;
    uint32_t *ki = key, *vi = val, *ko = key_alt, *vo = val_alt;
    int passes = (bits + kRadixBits - 1) / kRadixBits;
    for (int p = 0; p < passes; ++p) {
        int shift = p * kRadixBits;
        emit<KRadixCount>({ki, n, shift, tile_counts, ntiles}, (uint32_t)ntiles, st);
        emit<KDigitScan>({tile_counts, ntiles, digit_total}, kDigits, st);
        emit<KRadixScatter>({ki, vi, ko, vo, n, shift, tile_counts, ntiles, digit_total}, (uint32_t)ntiles, st);
        uint32_t *t = ki; ki = ko; ko = t;
        t = vi; vi = vo; vo = t;
    }
    // after an odd number of passes the sorted keys and values are in the alternate buffers
    return ki != key;
}

void launch_cell_ranges(const uint32_t *key_sorted, int64_t n, int64_t G, uint32_t *cell_start,
                        void *scratch, hipStream_t st)
{
    const int64_t ntiles = (n + kTile - 1) / kTile;
    uint32_t *run_start = (uint32_t *)scratch + (size_t)kDigits * (size_t)ntiles + kDigits;
    const int64_t nruns = G / kRangeBoxes + 1;
    emit<KRunStarts>({key_sorted, n, nruns, run_start}, grid1(n + 1), st);
    emit<KCellRanges>({key_sorted, G, run_start, cell_start}, (uint32_t)nruns, st);
}

void launch_cell_fixup(const uint32_t *key_sorted, int64_t n, uint32_t *val, const uint32_t *id_old,
                       hipStream_t st)
{
    emit<KCellFixup>({key_sorted, n, val, id_old}, grid1(n), st);
}

void launch_gather(PSet from, PSet to, const uint32_t *perm, int64_t n, hipStream_t st)
{
    emit<KGather>({from, to, perm, n}, grid1(n), st);
}

}  // namespace dcm
