// sort.hip -- binning of particles into storage cells by a counting sort (Section 4, Eq. 9-10).
//
// Each particle gets the key of its storage cell (its box, and the half of it along x; see
// cell_key). Particles are counted per cell with integer atomics, which also hand each one its
// rank among the particles of its cell; an exclusive scan of the counts gives the first slot of
// every cell, and each particle goes to its cell's first slot plus its rank. The ranks depend on
// the order in which the atomics land, so slots inside a cell are then ordered by particle id:
// the internal order -- and with it every summation order -- is a function of the state alone.
// The box counts b_ijk of Eq. 9 are sums of the differences of consecutive cell starts.
#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

constexpr int kBlockWaves = kBlock / 64;
constexpr int kScanPer = kCellScanBlock / kBlock;   // cells per thread of the cell scan
constexpr int kScanCells = kCellScanBlock;          // cells per scan block

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
    p.x = wrap_periodic(p.x, g.L[0]);
    p.y = wrap_periodic(p.y, g.L[1]);
    p.z = wrap_periodic(p.z, g.L[2]);
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

// Per-cell counts (cnt, zero on entry) and each particle's rank in its cell; bsum gets the
// number of particles in every block of kScanCells cells (one atomic per block present in a
// wave: the lanes of a wave that fall in one block are counted together). A workgroup takes
// kCountChunks consecutive chunks of kBlock particles, so that each wave has that many
// independent load-atomic-store chains in flight.
constexpr int kCountChunks = 4;

struct KCellCount {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        const uint32_t *key;
        int64_t n;
        uint32_t *cnt;
        uint32_t *rank;
        uint32_t *bsum;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        const int64_t i0 = (int64_t)blk * (kThreads * kCountChunks) + threadIdx.x;
        uint32_t k[kCountChunks];
        int64_t i[kCountChunks];
        bool valid[kCountChunks];
#pragma unroll
        for (int u = 0; u < kCountChunks; ++u) {
            i[u] = i0 + (int64_t)u * kThreads;
            valid[u] = i[u] < a.n;
            k[u] = valid[u] ? a.key[i[u]] : 0u;
        }
        count_cells<kCountChunks>(valid, k, i, a.cnt, a.rank, a.bsum);
    }
};

// cell_start[c] = particles in cells below c: each block scans its kScanCells counts and adds
// the particles of the blocks before it; the counts go back to zero. The block's counts pass
// through LDS so that global reads and writes are coalesced 16-byte accesses (four cells each)
// while each thread scans a run of kScanPer consecutive cells (rows padded by one word against
// bank conflicts). Both arrays start 256-byte aligned and blocks start at multiples of
// kScanCells, so every full group of four cells is one aligned 16-byte word.
struct KCellScan {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        uint32_t *cnt;
        uint32_t *cell_start;
        const uint32_t *bsum;   // particles per block of kScanCells cells
        int64_t ncells;     // key_count + 1 (the last start is the particle count)
        Grid g;
        uint32_t *image;    // optional: the box counts of Eq. 9 as an image in box order
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        static_assert(kScanPer % 4 == 0, "rows of whole 16-byte groups");
        constexpr int kQuads = kScanCells / 4 / kBlock;     // 16-byte groups per thread
        __shared__ uint32_t lds[kBlockWaves];
        __shared__ uint32_t tile[kBlock * (kScanPer + 1)];
        const int64_t base = (int64_t)blk * kScanCells;
        // coalesced load: group g (cells 4g .. 4g + 3 of the block) goes to row 4g / kScanPer
#pragma unroll
        for (int q = 0; q < kQuads; ++q) {
            const int gq = q * kBlock + threadIdx.x;
            const int64_t c = base + 4 * (int64_t)gq;
            uint32_t v[4] = {0u, 0u, 0u, 0u};
            if (c + 3 < a.ncells) {
                uint4 *w = (uint4 *)(a.cnt + c);
                const uint4 x = *w;
                v[0] = x.x; v[1] = x.y; v[2] = x.z; v[3] = x.w;
                // cleared for the next step (most groups of cells are empty)
                if (x.x | x.y | x.z | x.w) *w = make_uint4(0u, 0u, 0u, 0u);
            } else {
                for (int j = 0; j < 4; ++j)
                    if (c + j < a.ncells) {
                        v[j] = a.cnt[c + j];
                        if (v[j]) a.cnt[c + j] = 0u;
                    }
            }
            const int e = 4 * gq;
            uint32_t *t = tile + (e / kScanPer) * (kScanPer + 1) + e % kScanPer;
            t[0] = v[0]; t[1] = v[1]; t[2] = v[2]; t[3] = v[3];
        }
        __syncthreads();
        // The box counts (Eq. 9), when asked for: a box's 2^sx cells are keys 2^(sy + sz) apart
        // inside one aligned group of 2^(sx + sy + sz) keys, so every box lies in one block. The
        // reads of the counts here come before the scan below overwrites them (its first barrier
        // separates the two).
        if (a.image) {
            const Grid &g = a.g;
            const int gs = g.sy + g.sz;
            const uint32_t ncx = (uint32_t)g.n[0] << g.sx, rows_y = (uint32_t)g.n[1] >> g.sy;
            for (int t = threadIdx.x; t < (kScanCells >> g.sx); t += kBlock) {
                const int place = t & ((1 << gs) - 1);
                const int e0 = ((t >> gs) << (g.sx + gs)) + place;
                const int64_t k0 = base + e0;
                if (k0 + 1 >= a.ncells) continue;   // past the last cell
                uint32_t cb = 0;
                for (int j = 0; j < (1 << g.sx); ++j) {
                    const int e = e0 + (j << gs);
                    cb += tile[(e / kScanPer) * (kScanPer + 1) + e % kScanPer];
                }
                const uint32_t rest = (uint32_t)(k0 >> gs);
                const uint32_t xa = (rest % ncx) >> g.sx, rw = rest / ncx;
                const uint32_t yb = ((rw % rows_y) << g.sy) | ((uint32_t)place & ((1u << g.sy) - 1u));
                const uint32_t zc = ((rw / rows_y) << g.sz) | ((uint32_t)place >> g.sy);
                a.image[((int64_t)zc * g.n[1] + yb) * g.n[0] + xa] = cb;
            }
        }
        uint32_t *row = tile + threadIdx.x * (kScanPer + 1);
        uint32_t s = 0;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) s += row[q];
        uint32_t excl;
        block_exclusive_scan(s, &excl, lds);
        // the particles of the blocks before this one: the block counts are complete before
        // the scan starts, and a few thousand of them sit in L2
        uint32_t before = 0, ignored;
        for (uint32_t j = threadIdx.x; j < blk; j += 4 * kBlock) {
            // four loads in flight per round
            uint32_t v[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) v[u] = j + u * kBlock < blk ? a.bsum[j + u * kBlock] : 0u;
            before += (v[0] + v[1]) + (v[2] + v[3]);
        }
        before = block_exclusive_scan(before, &ignored, lds);
        uint32_t run = before + excl;
#pragma unroll
        for (int q = 0; q < kScanPer; ++q) {
            const uint32_t v = row[q];
            row[q] = run;
            run += v;
        }
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kQuads; ++q) {
            const int gq = q * kBlock + threadIdx.x;
            const int64_t c = base + 4 * (int64_t)gq;
            const int e = 4 * gq;
            const uint32_t *t = tile + (e / kScanPer) * (kScanPer + 1) + e % kScanPer;
            if (c + 3 < a.ncells) {
                *(uint4 *)(a.cell_start + c) = make_uint4(t[0], t[1], t[2], t[3]);
            } else {
                for (int j = 0; j < 4; ++j)
                    if (c + j < a.ncells) a.cell_start[c + j] = t[j];
            }
        }
    }
};

// Slot of particle i: its cell's start plus its rank; val_out records where it came from.
struct KCellScatter {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        const uint32_t *key;
        const uint32_t *rank;
        const uint32_t *cell_start;
        int64_t n;
        uint32_t *key_out;
        uint32_t *val_out;
        uint32_t *bsum;     // cleared here for the next count (the scan has read it)
        int64_t nb;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        const int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        if (i < a.nb) a.bsum[i] = 0u;
        if (i >= a.n) return;
        const uint32_t k = a.key[i];
        const uint32_t p = a.cell_start[k] + a.rank[i];
        a.key_out[p] = k;
        a.val_out[p] = (uint32_t)i;
    }
};

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
    // the three keys loaded together (no short circuit between the loads)
    const uint32_t k = key[s], kn = key[s + 1], kp = key[s > 0 ? s - 1 : s + 1];
    if ((s > 0 && kp == k) || kn != k) return;
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

// Scratch of the cell sort: per-cell counts [K + 1], ranks [n], per-block counts.
static int64_t scan_blocks(int64_t K) { return (K + 1 + kScanCells - 1) / kScanCells; }

size_t sort_scratch_bytes(int64_t n, int64_t K)
{
    return sizeof(uint32_t) * ((size_t)(K + 1) + (size_t)n + (size_t)scan_blocks(K));
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

void launch_cell_sort_init(void *scratch, int64_t n, int64_t K, hipStream_t st)
{
    uint32_t *cnt = (uint32_t *)scratch;
    uint32_t *bsum = cnt + (K + 1) + n;
    launch_fill_u32(cnt, 0u, K + 1, st);
    launch_fill_u32(bsum, 0u, scan_blocks(K), st);
}

CellCounts cell_sort_counts(void *scratch, int64_t n, int64_t K)
{
    uint32_t *cnt = (uint32_t *)scratch;
    return {cnt, cnt + (K + 1), cnt + (K + 1) + n};
}

void launch_cell_sort(const Grid &g, const uint32_t *key, uint32_t *key_out, uint32_t *val_out,
                      uint32_t *cell_start, void *scratch, int64_t n, bool counted, uint32_t *image, hipStream_t st)
{
    const int64_t K = key_count(g);
    uint32_t *cnt = (uint32_t *)scratch;
    uint32_t *rank = cnt + (K + 1);
    uint32_t *bsum = rank + n;
    const int64_t nb = scan_blocks(K);
    if (!counted)
        emit<KCellCount>({key, n, cnt, rank, bsum}, (uint32_t)((n + kBlock * kCountChunks - 1) / (kBlock * kCountChunks)), st);
    emit<KCellScan>({cnt, cell_start, bsum, K + 1, g, image}, (uint32_t)nb, st);
    const int64_t m = n > nb ? n : nb;
    emit<KCellScatter>({key, rank, cell_start, n, key_out, val_out, bsum, nb}, grid1(m), st);
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
