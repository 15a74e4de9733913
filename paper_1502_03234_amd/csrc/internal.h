// internal.h -- shared declarations of libdcm's HIP translation units (not part of the ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <climits>
#include <vector>
#include <cstdint>

#include "../../include/dcm.h"

namespace dcm {

constexpr int kBlock = 256;               // threads per workgroup for streaming kernels
constexpr int kHistBins = 65536;          // capacity of the smoothed-value histogram
constexpr uint32_t kInvalid = 0xFFFFFFFFu;

// sticky device condition bits (dcm_check)
constexpr uint32_t kFlagNonFinite = 1u;
constexpr uint32_t kFlagHistOverflow = 2u;
constexpr uint32_t kFlagNotConverged = 4u;
constexpr uint32_t kFlagBadCutoff = 8u;
constexpr uint32_t kFlagListOverflow = 16u;

// Grid geometry shared by every kernel that maps positions to boxes (Eq. 10).
struct Grid {
    int32_t n[3];       // N_x, N_y, N_z
    double h[3];        // box edges L_k / N_k
    double L[3];        // periodic box
    int64_t G;          // N_x N_y N_z
    int32_t sy, sz;     // log2 of the y and z extent of a force row (0 or 1; see cell_key)
    int32_t sx;         // log2 of the storage cells per box along x (0 or 1; see cell_key)
};

// Sort key (storage order) of storage cell (ax, b, c), where ax counts cells of h_x / 2^sx along
// x (box a holds cells a 2^sx .. a 2^sx + 2^sx - 1). Boxes are grouped into force rows of 2^sy x
// 2^sz boxes in y and z; keys run over force rows, then x cells, then the box's place inside its
// force row. The boxes of one force row and an x-interval (in cells) are therefore one
// contiguous key range; with sx = sy = sz = 0 the key is the plain linear box index
// (c N_y + b) N_x + a. The particles of box (a, b, c) are the 2^sx key ranges of its cells.
__host__ __device__ inline uint32_t cell_key(const Grid &g, int32_t ax, int32_t b, int32_t c)
{
    const uint32_t row = (uint32_t)(c >> g.sz) * (uint32_t)(g.n[1] >> g.sy) + (uint32_t)(b >> g.sy);
    const uint32_t sub = ((uint32_t)(c & ((1 << g.sz) - 1)) << g.sy) | (uint32_t)(b & ((1 << g.sy) - 1));
    return ((row * ((uint32_t)g.n[0] << g.sx) + (uint32_t)ax) << (g.sy + g.sz)) | sub;
}

// Number of storage keys (cells).
__host__ __device__ inline int64_t key_count(const Grid &g) { return g.G << g.sx; }

// Particles in box (a, b, c) (Eq. 9): the lengths of its cells' key ranges.
__device__ inline uint32_t box_count(const Grid &g, const uint32_t *cell_start, int32_t a, int32_t b, int32_t c)
{
    // the box's first cell, and its second one a force row of keys further on (sx = 1)
    const uint32_t k = cell_key(g, a << g.sx, b, c);
    uint32_t cnt = cell_start[k + 1] - cell_start[k];
    if (g.sx) {
        const uint32_t k2 = k + (1u << (g.sy + g.sz));
        cnt += cell_start[k2 + 1] - cell_start[k2];
    }
    return cnt;
}

// Box index of a wrapped coordinate along an axis of N boxes of edge h (Eq. 10: floor(x / h),
// clamped to 0 .. N - 1).
__host__ __device__ inline int32_t box_index(double x, double h, int32_t N)
{
    const double f = floor(x / h);
    int32_t i = (int32_t)f;
    if (f > (double)(N - 1)) i = N - 1;
    if (i < 0) i = 0;
    return i;
}

// Storage key of a wrapped position: its box (Eq. 10) and, inside the box, its x cell (used
// only to narrow the force kernel's x-intervals; the box alone decides the counts).
__host__ __device__ inline uint32_t pos_key(const Grid &g, double x, double y, double z)
{
    const int32_t a = box_index(x, g.h[0], g.n[0]);
    const int32_t b = box_index(y, g.h[1], g.n[1]);
    const int32_t c = box_index(z, g.h[2], g.n[2]);
    int32_t q = 0;
    if (g.sx) {
        const int32_t S = 1 << g.sx;
        const double f = floor(x * ((double)S / g.h[0])) - (double)a * S;
        q = f < 0.0 ? 0 : (f > (double)(S - 1) ? S - 1 : (int32_t)f);
    }
    return cell_key(g, (a << g.sx) + q, b, c);
}

// Cells per block of the cell-start scan (the counting sort's per-block counts are over these).
constexpr int kCellScanBlock = 4096;

// Counting step of the counting sort, for C chunks of consecutive particles held one per lane
// (i[u], key k[u], valid[u]; valid lanes are a prefix of the wave): cnt[k] counts the cell's
// particles, rank[i] gets the particle's place among them, bsum[k / kCellScanBlock] the
// block's count. Particles arrive nearly in cell order, so a run of neighbouring lanes with one
// key takes its ranks with one atomic of its first lane, and the lanes of a wave that fall in
// one block add to its count together. The C chunks' atomics are issued before any result is
// used. Every lane of the wave must call it.
template <int C>
__device__ __forceinline__ void count_cells(const bool (&valid)[C], const uint32_t (&k)[C], const int64_t (&i)[C],
                                            uint32_t *cnt, uint32_t *rank, uint32_t *bsum)
{
    const unsigned lane = __lane_id();
    uint32_t base[C];
    int leader[C];
#pragma unroll
    for (int u = 0; u < C; ++u) {
        const uint32_t prev = __shfl_up(k[u], 1, 64);
        const unsigned long long vmask = __ballot(valid[u]);
        const unsigned long long starts = __ballot(valid[u] && (lane == 0 || prev != k[u]));
        // this lane's run starts at the highest start at or below it, and ends at the next
        // start or the first invalid lane above that
        const unsigned long long upto = lane == 63 ? ~0ull : ((2ull << lane) - 1ull);
        const unsigned long long mine = starts & upto;
        leader[u] = mine ? 63 - __clzll((long long)mine) : (int)lane;
        const unsigned long long later = leader[u] == 63 ? 0ull : ~((2ull << leader[u]) - 1ull);
        const unsigned long long ends = (starts | ~vmask) & later;
        const int next = ends ? __ffsll((long long)ends) - 1 : 64;
        base[u] = 0u;
        if (valid[u] && lane == (unsigned)leader[u]) base[u] = atomicAdd(&cnt[k[u]], (uint32_t)(next - leader[u]));
    }
#pragma unroll
    for (int u = 0; u < C; ++u) {
        const uint32_t b = __shfl(base[u], valid[u] ? leader[u] : (int)lane, 64);
        if (valid[u]) rank[i[u]] = b + (lane - (unsigned)leader[u]);
        const uint32_t sb = k[u] / (uint32_t)kCellScanBlock;
        unsigned long long todo = __ballot(valid[u]);
        while (todo) {
            const int first = __ffsll((long long)todo) - 1;
            const uint32_t lb = __shfl(sb, first, 64);
            const unsigned long long peers = __ballot(valid[u] && sb == lb) & todo;
            if (lane == (unsigned)first) atomicAdd(&bsum[lb], (uint32_t)__popcll(peers));
            todo &= ~peers;
        }
    }
}

// A coordinate wrapped into the periodic box [0, L). Where rounding would leave the result
// outside (|x| so large that x - L floor(x / L) loses the fraction), it becomes 0, so that every
// position the kernels index cells with lies inside the box; NaN stays NaN.
__device__ __forceinline__ double wrap_periodic(double x, double L)
{
    double t = x - L * floor(x / L);
    if (t < 0.0) t += L;
    if (t < 0.0 || t >= L) t = 0.0;
    return t;
}

// One copy of the per-particle state in cell-sorted order.
struct PSet {
    double4 *pos;       // x, y, z, r_c
    double *vx, *vy, *vz;
    uint32_t *id;       // caller index of the particle in this slot
};

// Per-block partial sums written by the force and kick kernels, reduced in fixed order.
struct Partial {
    double e, w[6], ke;
    long long pairs;
    long long pad;
};

// Constants of the Nose-Hoover half step: time step, g T* (g = 3n - 3 degrees of freedom) and
// the thermostat mass Q = g T* tau^2.
struct NhConst {
    double dt, gT, Q;
};
enum { kNhNone = 0, kNhStart = 1, kNhEnd = 2 };

// Scratch of the grid pipeline (interface detection), G entries each unless noted.
// Box labels after segmentation (Eq. 11-12).
constexpr uint8_t kLabelLiquid = 0, kLabelVapor = 1;

// Working arrays of the Mumford-Shah segmentation (G boxes each; p holds 3 G).
struct MsWork {
    double *u, *ub, *p, *r;
};
struct MsParams {
    double nu;       // perimeter weight of Eq. 13 (0: plain threshold)
    double Lmax;     // longest box edge (the length unit of nu)
    int32_t iters;   // primal-dual iterations
};

struct GridWork {
    uint32_t *cell_start;   // [G + 1] first sorted slot of each box (Eq. 9 counts = differences)
    uint32_t *g;            // smoothed image
    uint32_t *gtmp;         // smoothing ping-pong
    uint8_t *raw;           // threshold labels
    uint8_t *label;         // labels after component removal
    uint32_t *parent;       // union-find parents (component = smallest member index)
    uint32_t *csize;        // component sizes (saturating at min_component)
    double *dist;           // box-interface distances
    uint32_t *hist;         // [kHistBins]
    double *km;             // [3] rho_v, rho_l, threshold
    long long *stats;       // [8] detection statistics
    uint32_t *changed;      // [max sweeps + 1] per-sweep change counters
    uint32_t *flags;        // [1] sticky device conditions
    uint32_t *tdirty;       // [2 * distance_tiles] pass flags of the distance tiles
    uint32_t *tcur;         // [2 * distance_tiles] which distance copy is current per tile
    double *dist2;          // second copy of the distance grid
    uint8_t *ctile;         // [component_tiles] tile kinds of the current component pass
    double *dist_v;         // box-liquid distances (tail correction only, else NULL)
    MsWork ms;              // Mumford-Shah segmentation (all NULL unless it is on)
};

// Records a message for dcm_last_error (printf format) and returns s.
dcm_status report_error(dcm_status s, const char *fmt, ...);

// ---- launchers (each enqueues on `st`; no synchronization) ------------------------------
// sort.hip
size_t sort_scratch_bytes(int64_t n, int64_t K);
void launch_wrap_key(const Grid &g, PSet s, int64_t n, uint32_t *key, uint32_t *val, hipStream_t st);
void launch_init_ids(PSet s, int64_t n, hipStream_t st);
// Box counts of the current positions into count (linear box index); clears count first.
void launch_count_boxes(const Grid &g, const double4 *pos, int64_t n, uint32_t *count, hipStream_t st);
// out[0] = max squared displacement since pos_build (minimum image), out[1] = max cutoff growth,
// as double bit patterns.
void launch_list_check(const Grid &g, const double4 *pos, const double4 *pos_build, int64_t n,
                       unsigned long long *out, hipStream_t st);
// Counting sort of the particles by storage-cell key (K = key_count cells): key_out / val_out
// get the keys in cell order and the source slot of each, cell_start [K + 1] the first slot of
// every cell. The sort's scratch holds per-cell counts that must be zero on entry: the sort
// leaves them zero, and launch_cell_sort_init zeroes them once for a new workspace.
void launch_cell_sort_init(void *scratch, int64_t n, int64_t K, hipStream_t st);
// counted = true: the keys' kernel has already counted them (cell_sort_counts) and the count
// step is skipped. image (optional, G words): also write the box counts of Eq. 9 there, in box
// order, as launch_count_from_ranges would from the cell starts.
void launch_cell_sort(const Grid &g, const uint32_t *key, uint32_t *key_out, uint32_t *val_out,
                      uint32_t *cell_start, void *scratch, int64_t n, bool counted, uint32_t *image,
                      hipStream_t st);
// The count, rank and block-count arrays inside the sort scratch, for a kernel that counts its
// keys as it writes them.
struct CellCounts {
    uint32_t *cnt, *rank, *bsum;
};
CellCounts cell_sort_counts(void *scratch, int64_t n, int64_t K);
void launch_cell_fixup(const uint32_t *key_sorted, int64_t n, uint32_t *val, const uint32_t *id_old,
                       hipStream_t st);
void launch_gather(PSet from, PSet to, const uint32_t *perm, int64_t n, hipStream_t st);

// detect.hip
void launch_smooth(const Grid &g, int passes, const uint32_t *cell_start, const uint32_t *in,
                   uint32_t *out, uint32_t *tmp, hipStream_t st);
// Two-means of the image's histogram (Eq. 14). The histogram is left at zero; hist_zero = true
// says it is zero on entry (a previous call on this workspace, or a zeroed new one).
void launch_two_means(const Grid &g, const uint32_t *img, GridWork w, long long *stats_out,
                      bool hist_zero, hipStream_t st);
// ms.nu > 0: Eq. 13's segmentation between the threshold and the component removal.
void launch_segment(const Grid &g, const uint32_t *img, const double *km, int32_t min_component,
                    const MsParams &ms, GridWork w, hipStream_t st);
// mumford_shah.hip: raw holds the threshold labels on entry; raw and label the segmentation's.
void launch_mumford_shah(const Grid &g, const uint32_t *img, const double *km, const MsParams &ms,
                         uint8_t *raw, uint8_t *label, MsWork m, hipStream_t st);
int max_distance_sweeps(const Grid &g, double cap);
int64_t distance_tiles(const Grid &g);
int64_t component_tiles(const Grid &g);

// Distance of every box to the boxes labelled `zero` (which get 0); the sweep count goes to
// *sweeps. The solve leaves its pass and tile flags at zero; flags_zero = true says they are
// zero already (a previous solve on this workspace, or launch_distance_flags_zero), so they
// are not cleared first.
void launch_distance(const Grid &g, double cap, const uint8_t *label, uint8_t zero, double *dist,
                     GridWork w, long long *sweeps, bool flags_zero, hipStream_t st);
void launch_distance_flags_zero(const Grid &g, double cap, GridWork w, hipStream_t st);
// dist_v (optional): box-liquid distances; the cutoff then takes the larger of the two depths.
void launch_cutoffs(const Grid &g, PSet s, int64_t n, const double *dist, const double *dist_v, double cap,
                    double rc_min, double rc_max, double alpha, double a, double b, int linear, hipStream_t st);
void launch_cap_copy(const double *dist, double cap, double *out, int64_t G, hipStream_t st);
void launch_count_from_ranges(const Grid &g, const uint32_t *cell_start, uint32_t *out, hipStream_t st);

// force.hip
struct ForceArgs {
    Grid grid;
    const double4 *pos;
    const uint32_t *cell_start;
    const uint32_t *id;
    int64_t n;
    double eps24, eps4, sigma2;
    double sigma6x2;        // 2 sigma^6 (the FP64 pair loop works in units of sigma^6)
    double eps24s6;         // 24 eps sigma^6
    float eps24f, sigma2f;  // the same constants for the FP32 precision form
    double rc_max;          // largest cutoff (search radius of the symmetric rule)
    int pair_rule;
    int energy_shift;
    int precision;
    double *fx, *fy, *fz;
    double *e_out;          // per-atom energy in caller order (optional)
    double *w_out;          // per-atom virial [6][n] in caller order (optional)
    uint32_t *pairs_out;    // per-atom pair count in caller order (optional)
    Partial *partials;      // [force_blocks(n)]
    uint32_t *flags;
    // neighbour lists (Verlet lists with a skin): list[k * n + i] is the k-th candidate slot
    // of slot i, nlist[i] their number; list_mode 1 evaluates forces from them
    int list_mode;
    uint32_t *list;
    uint32_t *nlist;
    uint32_t list_cap;
    // launch order of the force waves (a permutation of the workgroups, longest last duration
    // first) and each wave's duration in its last launch (constant-rate clock ticks); the
    // forces do not depend on the order
    uint32_t *order;
    uint32_t *wave_time;
    uint32_t *wave_hist;    // wave_order_scratch_words() words for the ordering
};
int force_blocks(int64_t n);
// The pair-force kernel alone; launch_force_wave_order then orders the waves for the next
// launch from the durations this one recorded (every force launch is followed by it).
void launch_forces(const ForceArgs &a, hipStream_t st);
void launch_force_wave_order(const ForceArgs &a, hipStream_t st);
// Longest-first order of nb force waves from their recorded durations.
size_t wave_order_scratch_words();
// counted = true: the force launch has already counted its waves into hist (which the
// ordering leaves at zero); false: count them from wave_time first (hist may hold anything).
void launch_wave_order(const uint32_t *wave_time, uint32_t *order, uint32_t *hist, int64_t nb, bool counted,
                       hipStream_t st);
// Lists of every slot within r_c[i] + skin, built by the force kernel's traversal (cell_start
// must describe the current positions); sets kFlagListOverflow if a list exceeds list_cap.
void launch_build_list(const ForceArgs &a, double skin, hipStream_t st);

// tail.hip
struct TailArgs {
    Grid grid;
    const double4 *pos;     // storage order, w = r_c
    const uint32_t *id;
    int64_t n;
    const double *dist_l;   // box-interface distances (vapor boxes 0)
    const double *dist_v;   // box-liquid distances (liquid boxes 0)
    const double *km;       // two-means centres {vapor, liquid, threshold} of the smoothed image
    double cap;             // distance band limit
    double half_edge;       // mean half box edge
    double inv_norm;        // 1 / (64^passes * box volume): centre -> number density
    double epsilon, sigma;
    double *fx, *fy, *fz;   // storage order, added to
    double *e_out;          // per-atom energy in caller order, added to (optional)
    Partial *partials;      // [force_blocks(n)] energy partials, added to
};
void launch_tail(const TailArgs &a, hipStream_t st);

// exact.hip
// Upper bound of the box visits of launch_forces_images (work guard).
double image_box_visits(const Grid &g, int64_t n, double R);
void launch_forces_images(const Grid &g, PSet s, const uint32_t *cell_start, int64_t n, double R,
                          double epsilon, double sigma, double *f_out, double *e_out, hipStream_t st);

// integrate.hip
void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st);
void launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st);
int stream_blocks(int64_t n);
// counts.cnt != nullptr: the kernel also takes the counting sort's count step on the keys it
// writes (the sort that follows is then launched with counted = true).
void launch_kick_drift_key(const Grid &g, PSet s, const double *fx, const double *fy,
                           const double *fz, int64_t n, double hdt, double dt, int second_kick,
                           const double *scale, uint32_t *key, CellCounts counts, Partial *ke_partials,
                           hipStream_t st);
void launch_kick(PSet s, const double *fx, const double *fy, const double *fz, int64_t n,
                 double hdt, Partial *ke_partials, hipStream_t st);
void launch_ke_only(PSet s, int64_t n, Partial *ke_partials, hipStream_t st);
void launch_scale(PSet s, int64_t n, const double *scale, Partial *ke_partials, hipStream_t st);
// Sums the partials into *out (optional); with nh_mode kNhStart/kNhEnd the final wave also takes
// half a thermostat step on nh = {xi, eta, scale} with the summed kinetic energy.
void launch_reduce_thermo(const Partial *force_parts, int nforce, const Partial *ke_parts, int nke,
                          double mass, long long step, dcm_thermo *out, Partial *stage, double *nh,
                          int nh_mode, const NhConst &c, hipStream_t st);
int reduce_stage_partials();
void launch_unsort(PSet s, const double *fx, const double *fy, const double *fz, int64_t n,
                   double *x_out, double *v_out, double *rc_out, double *f_out, hipStream_t st);
void launch_load_state(PSet s, const double *x, const double *v, const double *rc, int64_t n,
                       double rc_fill, hipStream_t st);
void launch_scatter_rc(PSet s, const double *rc_in, int64_t n, double rc_min, double rc_max,
                       uint32_t *flags, hipStream_t st);
void launch_check_finite(const double *a, int64_t count, uint32_t *flags, hipStream_t st);

}  // namespace dcm

// Handle of one system (shared by the C ABI and the serving loop).
namespace dcm {
struct Event {
    int stage;
    hipEvent_t a, b;
};
}  // namespace dcm

struct dcm_system {
    dcm_params p;
    int64_t n;
    dcm::Grid grid;
    double hdt, cut_a, cut_b, cap;
    dcm::PSet set[2];
    int cur;
    double *fx, *fy, *fz;
    uint32_t *key, *val, *key_alt, *val_alt;
    void *sort_scratch;
    dcm::GridWork gw;
    dcm::Partial *fparts, *kparts, *rparts;
    uint32_t *order, *wave_time;  // [nfb] force-wave launch order and last durations
    uint32_t *wave_hist;          // scratch of the wave ordering
    double *nh;             // Nose-Hoover state {xi, eta, velocity scale of the last half step}
    dcm::NhConst nhc;
    int nfb, nkb;
    int64_t k;
    int profiling;          // 0 off, 1 every stage, 2 the pair-force stage only
    bool stage_open;        // the current stage's start event was recorded
    std::vector<dcm::Event> events, spare;
    double ms[DCM_NSTAGES];
    int64_t counts[DCM_NSTAGES];
    // neighbour-list mode
    uint32_t *list, *nlist, list_cap;
    double4 *pos_build;          // positions and cutoffs at the last list build (storage order)
    uint32_t *box_count;         // box counts of the current positions
    unsigned long long *check;   // [2] list check results
    bool list_valid;
    int64_t list_builds;
};
