// api.cpp -- host side of the C ABI declared in include/dcm.h.
//
// Validates parameters, lays the caller's workspace out into the device arrays the kernels
// use, and enqueues the per-step sequence on the caller's stream. Nothing here allocates
// device memory; the only host allocations are the handle itself and profiling events.
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <string>
#include <utility>
#include <vector>

#include "internal.h"
#include "launch.h"

namespace dcm {

Recorder *&current_recorder()
{
    static thread_local Recorder *r = nullptr;
    return r;
}

}  // namespace dcm

using namespace dcm;

namespace {

// work guard of dcm_exact_forces (about a second of the image-sum kernel)
constexpr double kMaxImageBoxVisits = 4e10;

thread_local std::string g_last_error;

dcm_status fail(dcm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

}  // namespace

dcm_status dcm::report_error(dcm_status s, const char *fmt, ...)
{
    char buf[512];
    va_list ap;
    va_start(ap, fmt);
    vsnprintf(buf, sizeof buf, fmt, ap);
    va_end(ap);
    g_last_error = buf;
    return s;
}

namespace {

dcm_status hip_status(const char *where)
{
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return fail(DCM_E_HIP, "%s: %s", where, hipGetErrorString(e));
    return DCM_OK;
}

// Bump allocator over the caller's workspace (256-byte aligned sub-arrays).
struct Bump {
    uint8_t *base;
    size_t off = 0;
    explicit Bump(void *b) : base((uint8_t *)b) {}
    template <typename T>
    T *take(size_t count)
    {
        off = (off + 255) & ~(size_t)255;
        T *p = base ? (T *)(base + off) : nullptr;
        off += sizeof(T) * count;
        return p;
    }
};

bool grid_of(const dcm_params *p, Grid &g)
{
    for (int k = 0; k < 3; ++k) {
        if (!(p->box[k] > 0.0) || !(p->bin > 0.0) || !std::isfinite(p->box[k])) return false;
        double nk = std::round(p->box[k] / p->bin);
        if (!(nk < 1e6)) return false;
        int32_t N = (int32_t)nk;
        if (N < 3) N = 3;
        g.n[k] = N;
        g.h[k] = p->box[k] / (double)N;
        g.L[k] = p->box[k];
    }
    g.G = (int64_t)g.n[0] * g.n[1] * g.n[2];
    g.sy = g.sz = g.sx = 0;
    return true;
}

// Upper bound on the segmentation's iterations (two launches each per detection).
constexpr int32_t kMaxMsIters = 100000;

dcm_status validate(const dcm_params *p, int64_t n, Grid &g)
{
    if (!p) return fail(DCM_E_INVALID, "params is NULL");
    // the pair-force kernel reads positions through a buffer descriptor with 32-bit byte offsets
    if (n < 2 || n >= ((int64_t)1 << 26)) return fail(DCM_E_INVALID, "n = %lld outside [2, 2^26)", (long long)n);
    if (!grid_of(p, g)) return fail(DCM_E_INVALID, "box edges and bin must be positive and finite");
    if (g.G >= ((int64_t)1 << 31)) return fail(DCM_E_INVALID, "grid of %lld boxes is too large", (long long)g.G);
    if (!(p->rc_min > 0.0) || !(p->rc_min <= p->rc_max))
        return fail(DCM_E_INVALID, "need 0 < rc_min <= rc_max (got %g, %g)", p->rc_min, p->rc_max);
    if (p->neighbor_list != 0 && p->neighbor_list != 1) return fail(DCM_E_INVALID, "neighbor_list must be 0 or 1");
    if (p->neighbor_list && (!(p->skin > 0.0) || !std::isfinite(p->skin)))
        return fail(DCM_E_INVALID, "skin must be positive and finite (got %g)", p->skin);
    if (p->neighbor_list && p->pair_rule != DCM_PAIR_I)
        return fail(DCM_E_INVALID, "neighbour lists need pair_rule DCM_PAIR_I");
    if (p->neighbor_list && p->list_capacity < 0) return fail(DCM_E_INVALID, "list_capacity must be >= 0");
    // the largest search radius: r_c^max, or r_c^max + skin when lists are built
    const double reach = p->rc_max + (p->neighbor_list ? p->skin : 0.0);
    for (int k = 0; k < 3; ++k) {
        if (!(reach < 0.5 * p->box[k]))
            return fail(DCM_E_INVALID, "search radius %g (rc_max, plus the skin with lists) must be below half the box edge %g",
                        reach, p->box[k]);
        int need = 2 * (int)std::ceil(reach / g.h[k]) + 2;
        if (g.n[k] < need)
            return fail(DCM_E_INVALID, "axis %d has %d boxes; the cutoff stencil needs %d", k, g.n[k], need);
    }
    // force rows of two boxes in y and in z where the axis has an even box count and room for
    // the stencil in units of two boxes (a lane's rows then never meet the same storage row twice)
    g.sy = (g.n[1] % 2 == 0 && g.n[1] >= 2 * (int)std::ceil(reach / g.h[1]) + 6) ? 1 : 0;
    g.sz = (g.n[2] % 2 == 0 && g.n[2] >= 2 * (int)std::ceil(reach / g.h[2]) + 6) ? 1 : 0;
    // storage cells of half a box along x (the force kernel's x-intervals end at half boxes),
    // while the cell keys fit 31 bits
    g.sx = (g.G << 1) < ((int64_t)1 << 31) ? 1 : 0;
    if (p->cutoff_shape != DCM_CUTOFF_EXP && p->cutoff_shape != DCM_CUTOFF_LINEAR)
        return fail(DCM_E_INVALID, "unknown cutoff_shape");
    if (p->cutoff_shape == DCM_CUTOFF_EXP && p->alpha == 0.0 && p->rc_min != p->rc_max)
        return fail(DCM_E_INVALID, "alpha must be non-zero");
    if (!std::isfinite(p->alpha)) return fail(DCM_E_INVALID, "alpha must be finite");
    if (p->smooth_passes < 0 || p->smooth_passes > 4) return fail(DCM_E_INVALID, "smooth_passes must be 0..4");
    if (p->min_component < 0) return fail(DCM_E_INVALID, "min_component must be >= 0");
    if (p->detect_every < 0) return fail(DCM_E_INVALID, "detect_every must be >= 0");
    if (!(p->dt > 0.0) || !(p->mass > 0.0) || !(p->sigma > 0.0) || !(p->epsilon >= 0.0))
        return fail(DCM_E_INVALID, "dt, mass and sigma must be positive, epsilon non-negative");
    if (p->precision != DCM_FP64 && p->precision != DCM_FP32C) return fail(DCM_E_INVALID, "unknown precision");
    if (p->pair_rule != DCM_PAIR_I && p->pair_rule != DCM_PAIR_MAX) return fail(DCM_E_INVALID, "unknown pair_rule");
    if (p->thermostat != DCM_NVE && p->thermostat != DCM_NOSE_HOOVER) return fail(DCM_E_INVALID, "unknown thermostat");
    if (p->thermostat == DCM_NOSE_HOOVER &&
        (!(p->temperature > 0.0) || !(p->tdamp > 0.0) || !std::isfinite(p->temperature) || !std::isfinite(p->tdamp)))
        return fail(DCM_E_INVALID, "the thermostat needs temperature > 0 and tdamp > 0 (got %g, %g)",
                    p->temperature, p->tdamp);
    if (p->tail != 0 && p->tail != 1) return fail(DCM_E_INVALID, "tail must be 0 or 1");
    if (p->vapor_cutoff != 0 && p->vapor_cutoff != 1) return fail(DCM_E_INVALID, "vapor_cutoff must be 0 or 1");
    if (!(p->ms_nu >= 0.0) || !std::isfinite(p->ms_nu)) return fail(DCM_E_INVALID, "ms_nu must be finite and >= 0");
    if (p->ms_nu > 0.0 && (p->ms_iters < 1 || p->ms_iters > kMaxMsIters))
        return fail(DCM_E_INVALID, "ms_iters must be in [1, %d] (got %d)", kMaxMsIters, p->ms_iters);
    if (p->tail && (p->pair_rule != DCM_PAIR_I || p->energy_shift))
        return fail(DCM_E_INVALID, "the tail correction needs pair_rule DCM_PAIR_I and energy_shift 0");
    return DCM_OK;
}

}  // namespace



namespace {

// Lays the system's arrays over `ws` (or only measures when ws is NULL).
size_t layout(dcm_system *s, void *ws)
{
    Bump b(ws);
    const int64_t n = s->n, G = s->grid.G;
    for (int q = 0; q < 2; ++q) {
        s->set[q].pos = b.take<double4>(n);
        s->set[q].vx = b.take<double>(n);
        s->set[q].vy = b.take<double>(n);
        s->set[q].vz = b.take<double>(n);
        s->set[q].id = b.take<uint32_t>(n);
    }
    s->fx = b.take<double>(n);
    s->fy = b.take<double>(n);
    s->fz = b.take<double>(n);
    s->key = b.take<uint32_t>(n);
    s->val = b.take<uint32_t>(n);
    s->key_alt = b.take<uint32_t>(n);
    s->val_alt = b.take<uint32_t>(n);
    s->sort_scratch = b.take<uint8_t>(sort_scratch_bytes(n, key_count(s->grid)));
    s->gw.cell_start = b.take<uint32_t>(key_count(s->grid) + 1);
    s->gw.g = b.take<uint32_t>(G);
    s->gw.gtmp = b.take<uint32_t>(G);
    s->gw.raw = b.take<uint8_t>(G);
    s->gw.label = b.take<uint8_t>(G);
    s->gw.parent = b.take<uint32_t>(G);
    s->gw.csize = b.take<uint32_t>(G);
    s->gw.dist = b.take<double>(G);
    s->gw.hist = b.take<uint32_t>(kHistBins);
    s->gw.km = b.take<double>(3);
    s->gw.stats = b.take<long long>(8);
    s->gw.changed = b.take<uint32_t>(max_distance_sweeps(s->grid, s->cap) + 1);
    s->gw.flags = b.take<uint32_t>(1);
    s->gw.tdirty = b.take<uint32_t>(2 * distance_tiles(s->grid));
    s->gw.tcur = b.take<uint32_t>(2 * distance_tiles(s->grid));
    s->gw.dist2 = b.take<double>(G);
    s->gw.ctile = b.take<uint8_t>(component_tiles(s->grid));
    s->gw.dist_v = (s->p.tail || s->p.vapor_cutoff) ? b.take<double>(G) : nullptr;
    s->gw.ms = MsWork{nullptr, nullptr, nullptr, nullptr};
    if (s->p.ms_nu > 0.0) {
        s->gw.ms.u = b.take<double>(G);
        s->gw.ms.ub = b.take<double>(G);
        s->gw.ms.p = b.take<double>(3 * G);
        s->gw.ms.r = b.take<double>(G);
    }
    s->list = s->nlist = nullptr;
    s->pos_build = nullptr;
    s->box_count = nullptr;
    s->check = nullptr;
    s->list_cap = 0;
    if (s->p.neighbor_list) {
        const double R = s->p.rc_max + s->p.skin;
        s->list_cap = s->p.list_capacity > 0 ? (uint32_t)s->p.list_capacity
                                             : (uint32_t)std::ceil(1.25 * 4.0 / 3.0 * M_PI * R * R * R);
        s->list = b.take<uint32_t>((int64_t)s->list_cap * n);
        s->nlist = b.take<uint32_t>(n);
        s->pos_build = b.take<double4>(n);
        s->box_count = b.take<uint32_t>(G);
        s->check = b.take<unsigned long long>(2);
    }
    s->nfb = force_blocks(n);
    s->nkb = stream_blocks(n);
    s->fparts = b.take<Partial>(s->nfb);
    s->order = b.take<uint32_t>(s->nfb);
    s->wave_time = b.take<uint32_t>(s->nfb);
    s->wave_hist = b.take<uint32_t>((int64_t)wave_order_scratch_words());
    s->kparts = b.take<Partial>(s->nkb);
    s->rparts = b.take<Partial>(reduce_stage_partials());
    s->nh = b.take<double>(4);
    return b.off + 256;
}

void init_derived(dcm_system *s)
{
    const dcm_params &p = s->p;
    s->hdt = 0.5 * p.dt / p.mass;
    double hmax = std::max(s->grid.h[0], std::max(s->grid.h[1], s->grid.h[2]));
    // the distance band ends a box beyond r_c^max, where the cutoff function is flat; the tail
    // correction sees the interface to 2 r_c^max and a box
    s->cap = (p.tail ? 2.0 * p.rc_max : p.rc_max) + hmax;
    if (p.rc_min != p.rc_max && p.cutoff_shape == DCM_CUTOFF_EXP) {
        s->cut_a = (p.rc_max - p.rc_min) / (std::exp2(p.alpha * p.rc_max) - 1.0);
        s->cut_b = p.rc_min - s->cut_a;
    } else {
        s->cut_a = 0.0;
        s->cut_b = p.rc_max;
    }
    // g = 3n - 3: the thermostat leaves the total momentum unchanged (it scales it), so the
    // centre-of-mass degrees of freedom are not thermalised
    const double g = 3.0 * (double)s->n - 3.0;
    s->nhc.dt = p.dt;
    s->nhc.gT = g * p.temperature;
    s->nhc.Q = g * p.temperature * p.tdamp * p.tdamp;
}

void stage_begin(dcm_system *s, int stage, hipStream_t st)
{
    s->stage_open = false;
    if (s->profiling == 0 || (s->profiling == 2 && stage != 7)) return;
    s->stage_open = true;
    Event e;
    if (!s->spare.empty()) { e = s->spare.back(); s->spare.pop_back(); }
    else { (void)hipEventCreate(&e.a); (void)hipEventCreate(&e.b); }
    e.stage = stage;
    (void)hipEventRecord(e.a, st);
    s->events.push_back(e);
}

void stage_end(dcm_system *s, hipStream_t st)
{
    if (!s->stage_open) return;
    s->stage_open = false;
    (void)hipEventRecord(s->events.back().b, st);
}

// Re-bin the current set after its keys were written: sort, box ranges, in-box id order, and
// gather into the other set.
// The count step of the counting sort inside the kick/drift kernel, on steps that re-bin
// (without neighbour lists every step re-bins; with them only a list rebuild does, from keys of
// its own).
CellCounts step_counts(const dcm_system *s)
{
    if (s->p.neighbor_list) return {nullptr, nullptr, nullptr};
    return cell_sort_counts(s->sort_scratch, s->n, key_count(s->grid));
}

// The buffer in which the smoothing passes expect the box-count image (launch_smooth puts it
// where the first pass does not write).
uint32_t *count_image_target(const dcm_system *s)
{
    const int passes = s->p.smooth_passes;
    return (passes > 0 && passes % 2 == 1) ? s->gw.gtmp : s->gw.g;
}

// image (optional): the sort also writes the box-count image there (a detection follows).
void rebin_sorted(dcm_system *s, hipStream_t st, bool counted = false, uint32_t *image = nullptr)
{
    PSet from = s->set[s->cur], to = s->set[1 - s->cur];
    launch_cell_sort(s->grid, s->key, s->key_alt, s->val_alt, s->gw.cell_start, s->sort_scratch, s->n, counted,
                     image, st);
    std::swap(s->key, s->key_alt);
    std::swap(s->val, s->val_alt);
    launch_cell_fixup(s->key, s->n, s->val, from.id, st);
    launch_gather(from, to, s->val, s->n, st);
    s->cur = 1 - s->cur;
}

// The detection stages; with_cutoffs = false leaves the cutoffs as they are (the tail
// correction of a state resumed between detections needs only the distance fields).
// counted = true: the sort just before wrote the box-count image (count_image_target).
void detect(dcm_system *s, hipStream_t st, bool with_cutoffs = true, bool counted = false)
{
    const Grid &g = s->grid;
    GridWork w = s->gw;
    stage_begin(s, 2, st);
    if (s->p.neighbor_list) {
        // particles keep their storage order between list builds: count the current positions
        launch_count_boxes(g, s->set[s->cur].pos, s->n, s->box_count, st);
        launch_smooth(g, s->p.smooth_passes, nullptr, s->box_count, w.g, w.gtmp, st);
    } else if (counted) {
        launch_smooth(g, s->p.smooth_passes, nullptr, count_image_target(s), w.g, w.gtmp, st);
    } else {
        launch_smooth(g, s->p.smooth_passes, w.cell_start, nullptr, w.g, w.gtmp, st);
    }
    stage_end(s, st);
    stage_begin(s, 3, st);
    launch_fill_u32((uint32_t *)w.stats, 0u, 16, st);
    launch_two_means(g, w.g, w, w.stats, true, st);
    stage_end(s, st);
    stage_begin(s, 4, st);
    MsParams ms = {s->p.ms_nu, std::max(s->p.box[0], std::max(s->p.box[1], s->p.box[2])), s->p.ms_iters};
    launch_segment(g, w.g, w.km, s->p.min_component, ms, w, st);
    stage_end(s, st);
    stage_begin(s, 5, st);
    launch_distance(g, s->cap, w.label, kLabelVapor, w.dist, w, w.stats + 5, true, st);
    if (w.dist_v) launch_distance(g, s->cap, w.label, kLabelLiquid, w.dist_v, w, w.stats + 6, true, st);
    stage_end(s, st);
    if (!with_cutoffs) return;
    stage_begin(s, 6, st);
    launch_cutoffs(g, s->set[s->cur], s->n, w.dist, s->p.vapor_cutoff ? w.dist_v : nullptr, s->cap,
                   s->p.rc_min, s->p.rc_max, s->p.alpha,
                   s->cut_a, s->cut_b, s->p.cutoff_shape == DCM_CUTOFF_LINEAR ? 1 : 0, st);
    stage_end(s, st);
}

// Arguments of the pair-force kernels (and the list build) for the current set.
ForceArgs force_args(const dcm_system *s, double *e_out, double *w_out, uint32_t *pairs_out)
{
    ForceArgs a;
    a.grid = s->grid;
    a.pos = s->set[s->cur].pos;
    a.cell_start = s->gw.cell_start;
    a.id = s->set[s->cur].id;
    a.n = s->n;
    a.eps24 = 24.0 * s->p.epsilon;
    a.eps4 = 4.0 * s->p.epsilon;
    a.sigma2 = s->p.sigma * s->p.sigma;
    {
        const double s6 = a.sigma2 * a.sigma2 * a.sigma2;
        a.sigma6x2 = 2.0 * s6;
        a.eps24s6 = a.eps24 * s6;
    }
    a.eps24f = (float)a.eps24;
    a.sigma2f = (float)a.sigma2;
    a.rc_max = s->p.rc_max;
    a.pair_rule = s->p.pair_rule;
    a.energy_shift = s->p.energy_shift;
    a.precision = s->p.precision;
    a.fx = s->fx;
    a.fy = s->fy;
    a.fz = s->fz;
    a.e_out = e_out;
    a.w_out = w_out;
    a.pairs_out = pairs_out;
    a.partials = s->fparts;
    a.flags = s->gw.flags;
    a.list_mode = s->p.neighbor_list;
    a.list = s->list;
    a.nlist = s->nlist;
    a.list_cap = s->list_cap;
    a.order = s->order;
    a.wave_time = s->wave_time;
    a.wave_hist = s->wave_hist;
    return a;
}

void forces(dcm_system *s, hipStream_t st, double *e_out, double *w_out, uint32_t *pairs_out)
{
    const ForceArgs a = force_args(s, e_out, w_out, pairs_out);
    stage_begin(s, 7, st);
    launch_forces(a, st);
    stage_end(s, st);
    stage_begin(s, 8, st);
    launch_force_wave_order(a, st);
    stage_end(s, st);
    if (s->p.tail) {
        TailArgs t;
        t.grid = s->grid;
        t.pos = a.pos;
        t.id = a.id;
        t.n = s->n;
        t.dist_l = s->gw.dist;
        t.dist_v = s->gw.dist_v;
        t.km = s->gw.km;
        t.cap = s->cap;
        t.half_edge = (s->grid.h[0] + s->grid.h[1] + s->grid.h[2]) / 6.0;
        t.inv_norm = 1.0 / (std::pow(64.0, s->p.smooth_passes) * s->grid.h[0] * s->grid.h[1] * s->grid.h[2]);
        t.epsilon = s->p.epsilon;
        t.sigma = s->p.sigma;
        t.fx = s->fx;
        t.fy = s->fy;
        t.fz = s->fz;
        t.e_out = e_out;
        t.partials = s->fparts;
        stage_begin(s, 9, st);
        launch_tail(t, st);
        stage_end(s, st);
    }
}

// Neighbour lists (Alg. 3.3 with a skin r_s). A list holds every slot within r_c[i] + r_s of
// slot i at its build. A pair within r_c[i] now was within r_c[i] + 2 D at the build (D = the
// largest displacement since), so every list still holds all its pairs while
// 2 D + max_i (r_c[i] - r_c[i] at the build) <= r_s. The host reads the two maxima once per
// step; a rebuild re-sorts the particles by box (the traversal reads box ranges) and records
// the positions and cutoffs it was built from.
dcm_status list_update(dcm_system *s, hipStream_t st, bool force_rebuild)
{
    stage_begin(s, 10, st);
    bool rebuild = force_rebuild || !s->list_valid;
    if (!rebuild) {
        launch_list_check(s->grid, s->set[s->cur].pos, s->pos_build, s->n, s->check, st);
        unsigned long long h[2] = {0, 0};
        (void)hipMemcpyAsync(h, s->check, sizeof h, hipMemcpyDeviceToHost, st);
        if (hipStreamSynchronize(st) != hipSuccess) { stage_end(s, st); return hip_status("neighbour-list check"); }
        double d2, grow;
        std::memcpy(&d2, &h[0], sizeof d2);
        std::memcpy(&grow, &h[1], sizeof grow);
        rebuild = !(2.0 * std::sqrt(d2) + grow <= s->p.skin);
    }
    if (rebuild) {
        launch_wrap_key(s->grid, s->set[s->cur], s->n, s->key, s->val, st);
        rebin_sorted(s, st);
        launch_build_list(force_args(s, nullptr, nullptr, nullptr), s->p.skin, st);
        launch_copy_bytes(s->pos_build, s->set[s->cur].pos, sizeof(double4) * (size_t)s->n, st);
        s->list_valid = true;
        s->list_builds += 1;
        uint32_t flags = 0;
        (void)hipMemcpyAsync(&flags, s->gw.flags, sizeof flags, hipMemcpyDeviceToHost, st);
        if (hipStreamSynchronize(st) != hipSuccess) { stage_end(s, st); return hip_status("neighbour-list build"); }
        if (flags & kFlagListOverflow) {
            s->list_valid = false;
            stage_end(s, st);
            return fail(DCM_E_INVALID, "a neighbour list exceeds list_capacity = %u slots", s->list_cap);
        }
    }
    stage_end(s, st);
    return DCM_OK;
}

dcm_status create_impl(const dcm_params *p, int64_t n, void *d_ws, size_t ws_bytes, const double *d_x,
                       const double *d_v, const double *d_rc, int64_t step, bool from_state,
                       dcm_stream_t stream, dcm_system **out)
{
    if (!out) return fail(DCM_E_INVALID, "out is NULL");
    Grid g;
    dcm_status rs = validate(p, n, g);
    if (rs != DCM_OK) return rs;
    if (!d_x || !d_v || (from_state && !d_rc)) return fail(DCM_E_INVALID, "state pointer is NULL");
    if (from_state && step < 0) return fail(DCM_E_INVALID, "step must be >= 0");
    dcm_system *s = new (std::nothrow) dcm_system();
    if (!s) return fail(DCM_E_INVALID, "out of host memory");
    s->p = *p;
    s->n = n;
    s->grid = g;
    init_derived(s);
    size_t need = layout(s, nullptr);
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < need) {
        delete s;
        return fail(DCM_E_WORKSPACE, "workspace needs %zu bytes, 256-byte aligned (got %zu at %p)", need,
                    ws_bytes, d_ws);
    }
    layout(s, d_ws);
    s->cur = 0;
    s->k = from_state ? step : 0;
    hipStream_t st = (hipStream_t)stream;
    launch_fill_u32(s->gw.flags, 0u, 1, st);
    launch_distance_flags_zero(s->grid, s->cap, s->gw, st);
    launch_cell_sort_init(s->sort_scratch, n, key_count(s->grid), st);
    launch_fill_u32(s->gw.hist, 0u, kHistBins, st);
    launch_fill_u32((uint32_t *)s->nh, 0u, 8, st);
    launch_fill_u32(s->wave_time, 0u, s->nfb, st);
    launch_wave_order(s->wave_time, s->order, s->wave_hist, s->nfb, false, st);
    launch_check_finite(d_x, 3 * n, s->gw.flags, st);
    launch_check_finite(d_v, 3 * n, s->gw.flags, st);
    launch_load_state(s->set[0], d_x, d_v, from_state ? d_rc : nullptr, n, p->rc_max, st);
    if (from_state) launch_scatter_rc(s->set[0], d_rc, n, p->rc_min, p->rc_max, s->gw.flags, st);
    launch_wrap_key(s->grid, s->set[0], n, s->key, s->val, st);
    rebin_sorted(s, st);
    bool redetect = !from_state || (p->detect_every > 0 && step % p->detect_every == 0);
    if (redetect) detect(s, st);
    else if (p->tail) detect(s, st, false);
    s->list_valid = false;
    s->list_builds = 0;
    if (p->neighbor_list) {
        dcm_status lr = list_update(s, st, true);
        if (lr != DCM_OK) { delete s; return lr; }
    }
    forces(s, st, nullptr, nullptr, nullptr);
    uint32_t flags = 0;
    (void)hipMemcpyAsync(&flags, s->gw.flags, sizeof flags, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) {
        delete s;
        return fail(DCM_E_HIP, "dcm_create: %s", hipGetErrorString(e));
    }
    rs = hip_status("dcm_create");
    if (rs != DCM_OK) { delete s; return rs; }
    if (flags & kFlagNonFinite) {
        delete s;
        return fail(DCM_E_NONFINITE, "non-finite coordinate, velocity or initial force");
    }
    if (flags & kFlagBadCutoff) {
        delete s;
        return fail(DCM_E_INVALID, "a cutoff lies outside [rc_min, rc_max]");
    }
    *out = s;
    return DCM_OK;
}

// Thermostatted steps: each is U_NH(dt/2) kick drift [re-bin, detect, forces] kick U_NH(dt/2).
// The opening half uses the kinetic energy of the velocities in memory (a pass of its own on the
// first step of a call, else the one fused into the previous step's closing scaling), so a run
// split over several calls, or resumed from a checkpoint, takes the same bits as one call.
dcm_status step_nose_hoover(dcm_system *s, int32_t nsteps, hipStream_t st, dcm_thermo *d_th)
{
    for (int32_t q = 1; q <= nsteps; ++q) {
        s->k += 1;
        stage_begin(s, 8, st);
        if (q == 1) launch_ke_only(s->set[s->cur], s->n, s->kparts, st);
        launch_reduce_thermo(s->fparts, 0, s->kparts, s->nkb, s->p.mass, s->k, nullptr, s->rparts, s->nh,
                             kNhStart, s->nhc, st);
        stage_end(s, st);
        stage_begin(s, 0, st);
        launch_kick_drift_key(s->grid, s->set[s->cur], s->fx, s->fy, s->fz, s->n, s->hdt, s->p.dt, 0,
                              s->nh + 2, s->key, step_counts(s), s->kparts, st);
        stage_end(s, st);
        const bool det = s->p.detect_every > 0 && s->k % s->p.detect_every == 0;
        if (!s->p.neighbor_list) {
            stage_begin(s, 1, st);
            rebin_sorted(s, st, true, det ? count_image_target(s) : nullptr);
            stage_end(s, st);
        }
        if (det) detect(s, st, true, !s->p.neighbor_list);
        if (s->p.neighbor_list) {
            dcm_status lr = list_update(s, st, false);
            if (lr != DCM_OK) return lr;
        }
        forces(s, st, nullptr, nullptr, nullptr);
        stage_begin(s, 0, st);
        launch_kick(s->set[s->cur], s->fx, s->fy, s->fz, s->n, s->hdt, s->kparts, st);
        stage_end(s, st);
        stage_begin(s, 8, st);
        launch_reduce_thermo(s->fparts, s->nfb, s->kparts, s->nkb, s->p.mass, s->k,
                             d_th ? d_th + (q - 1) : nullptr, s->rparts, s->nh, kNhEnd, s->nhc, st);
        stage_end(s, st);
        stage_begin(s, 0, st);
        launch_scale(s->set[s->cur], s->n, s->nh + 2, s->kparts, st);
        stage_end(s, st);
    }
    return DCM_OK;
}

}  // namespace

extern "C" {

const char *dcm_version(void) { return "dcm-mi355x 0.1 (gfx950)"; }

const char *dcm_last_error(void) { return g_last_error.c_str(); }

dcm_status dcm_grid_dims(const dcm_params *p, int32_t dims[3])
{
    if (!p || !dims) return fail(DCM_E_INVALID, "NULL argument");
    Grid g;
    if (!grid_of(p, g)) return fail(DCM_E_INVALID, "box edges and bin must be positive and finite");
    for (int k = 0; k < 3; ++k) dims[k] = g.n[k];
    return DCM_OK;
}

dcm_status dcm_workspace_bytes(const dcm_params *p, int64_t n, size_t *bytes)
{
    if (!bytes) return fail(DCM_E_INVALID, "bytes is NULL");
    Grid g;
    dcm_status rs = validate(p, n, g);
    if (rs != DCM_OK) return rs;
    dcm_system tmp;
    tmp.p = *p;
    tmp.n = n;
    tmp.grid = g;
    init_derived(&tmp);
    *bytes = layout(&tmp, nullptr);
    return DCM_OK;
}

dcm_status dcm_create(const dcm_params *p, int64_t n, void *d_ws, size_t ws_bytes, const double *d_x,
                      const double *d_v, dcm_stream_t stream, dcm_system **out)
{
    return create_impl(p, n, d_ws, ws_bytes, d_x, d_v, nullptr, 0, false, stream, out);
}

dcm_status dcm_create_from_state(const dcm_params *p, int64_t n, void *d_ws, size_t ws_bytes,
                                 const double *d_x, const double *d_v, const double *d_rc,
                                 int64_t step, dcm_stream_t stream, dcm_system **out)
{
    return create_impl(p, n, d_ws, ws_bytes, d_x, d_v, d_rc, step, true, stream, out);
}

dcm_status dcm_set_cutoffs(dcm_system *s, dcm_stream_t stream, const double *d_rc)
{
    if (!s || !d_rc) return fail(DCM_E_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    launch_scatter_rc(s->set[s->cur], d_rc, s->n, s->p.rc_min, s->p.rc_max, s->gw.flags, st);
    if (s->p.neighbor_list) {
        dcm_status lr = list_update(s, st, false);
        if (lr != DCM_OK) return lr;
    }
    forces(s, st, nullptr, nullptr, nullptr);
    return hip_status("dcm_set_cutoffs");
}

dcm_status dcm_detect_interface(dcm_system *s, dcm_stream_t stream, const dcm_detect_out *o)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    if (o && o->dist_v && !s->gw.dist_v)
        return fail(DCM_E_INVALID, "dist_v needs tail = 1 or vapor_cutoff = 1");
    hipStream_t st = (hipStream_t)stream;
    detect(s, st);
    if (s->p.neighbor_list) {
        // the new cutoffs may have outgrown the lists
        dcm_status lr = list_update(s, st, false);
        if (lr != DCM_OK) return lr;
    }
    if (o) {
        const int64_t G = s->grid.G;
        if (o->count) {
            if (s->p.neighbor_list) launch_copy_bytes(o->count, s->box_count, sizeof(uint32_t) * (size_t)G, st);
            else launch_count_from_ranges(s->grid, s->gw.cell_start, o->count, st);
        }
        if (o->smooth) launch_copy_bytes(o->smooth, s->gw.g, sizeof(uint32_t) * G, st);
        if (o->raw) launch_copy_bytes(o->raw, s->gw.raw, (size_t)G, st);
        if (o->label) launch_copy_bytes(o->label, s->gw.label, (size_t)G, st);
        if (o->dist) launch_cap_copy(s->gw.dist, s->cap, o->dist, G, st);
        if (o->rc) launch_unsort(s->set[s->cur], s->fx, s->fy, s->fz, s->n, nullptr, nullptr, o->rc, nullptr, st);
        if (o->km) launch_copy_bytes(o->km, s->gw.km, 3 * sizeof(double), st);
        if (o->stats) launch_copy_bytes(o->stats, s->gw.stats, 6 * sizeof(long long), st);
        if (o->dist_v) launch_cap_copy(s->gw.dist_v, s->cap, o->dist_v, G, st);
    }
    return hip_status("dcm_detect_interface");
}

dcm_status dcm_compute_forces(dcm_system *s, dcm_stream_t stream, double *d_f, double *d_e, double *d_w,
                              uint32_t *d_pairs, dcm_thermo *d_th)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    hipStream_t st = (hipStream_t)stream;
    forces(s, st, d_e, d_w, d_pairs);
    if (d_f) launch_unsort(s->set[s->cur], s->fx, s->fy, s->fz, s->n, nullptr, nullptr, nullptr, d_f, st);
    if (d_th) {
        launch_ke_only(s->set[s->cur], s->n, s->kparts, st);
        launch_reduce_thermo(s->fparts, s->nfb, s->kparts, s->nkb, s->p.mass, s->k, d_th, s->rparts, s->nh,
                             kNhNone, s->nhc, st);
    }
    return hip_status("dcm_compute_forces");
}

dcm_status dcm_exact_forces(dcm_system *s, double R, dcm_stream_t stream, double *d_f, double *d_e)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    if (!(R > 0.0) || !std::isfinite(R)) return fail(DCM_E_INVALID, "R must be positive and finite");
    if (image_box_visits(s->grid, s->n, R) > kMaxImageBoxVisits)
        return fail(DCM_E_INVALID, "R = %g needs more than %.0e box visits for %lld particles", R,
                    kMaxImageBoxVisits, (long long)s->n);
    if (!d_f && !d_e) return DCM_OK;
    launch_forces_images(s->grid, s->set[s->cur], s->gw.cell_start, s->n, R, s->p.epsilon, s->p.sigma, d_f,
                         d_e, (hipStream_t)stream);
    return hip_status("dcm_exact_forces");
}

dcm_status dcm_step(dcm_system *s, int32_t nsteps, dcm_stream_t stream, dcm_thermo *d_th)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    if (nsteps < 0) return fail(DCM_E_INVALID, "nsteps must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    if (s->p.thermostat == DCM_NOSE_HOOVER) {
        dcm_status rs = step_nose_hoover(s, nsteps, st, d_th);
        if (rs != DCM_OK) return rs;
        return hip_status("dcm_step");
    }
    for (int32_t q = 1; q <= nsteps; ++q) {
        s->k += 1;
        stage_begin(s, 0, st);
        launch_kick_drift_key(s->grid, s->set[s->cur], s->fx, s->fy, s->fz, s->n, s->hdt, s->p.dt,
                              q > 1 ? 1 : 0, nullptr, s->key, step_counts(s), s->kparts, st);
        stage_end(s, st);
        if (q > 1 && d_th) {
            stage_begin(s, 8, st);
            launch_reduce_thermo(s->fparts, s->nfb, s->kparts, s->nkb, s->p.mass, s->k - 1, d_th + (q - 2),
                                 s->rparts, s->nh, kNhNone, s->nhc, st);
            stage_end(s, st);
        }
        const bool det = s->p.detect_every > 0 && s->k % s->p.detect_every == 0;
        if (!s->p.neighbor_list) {
            stage_begin(s, 1, st);
            rebin_sorted(s, st, true, det ? count_image_target(s) : nullptr);
            stage_end(s, st);
        }
        if (det) detect(s, st, true, !s->p.neighbor_list);
        if (s->p.neighbor_list) {
            dcm_status lr = list_update(s, st, false);
            if (lr != DCM_OK) return lr;
        }
        forces(s, st, nullptr, nullptr, nullptr);
    }
    if (nsteps > 0) {
        stage_begin(s, 0, st);
        launch_kick(s->set[s->cur], s->fx, s->fy, s->fz, s->n, s->hdt, s->kparts, st);
        stage_end(s, st);
        if (d_th) {
            stage_begin(s, 8, st);
            launch_reduce_thermo(s->fparts, s->nfb, s->kparts, s->nkb, s->p.mass, s->k, d_th + (nsteps - 1),
                                 s->rparts, s->nh, kNhNone, s->nhc, st);
            stage_end(s, st);
        }
    }
    return hip_status("dcm_step");
}

dcm_status dcm_get_thermostat(dcm_system *s, dcm_stream_t stream, double h_xi_eta[2])
{
    if (!s || !h_xi_eta) return fail(DCM_E_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    double t[2];
    (void)hipMemcpyAsync(t, s->nh, sizeof t, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(DCM_E_HIP, "dcm_get_thermostat: %s", hipGetErrorString(e));
    h_xi_eta[0] = t[0];
    h_xi_eta[1] = t[1];
    return hip_status("dcm_get_thermostat");
}

dcm_status dcm_set_thermostat(dcm_system *s, dcm_stream_t stream, const double h_xi_eta[2])
{
    if (!s || !h_xi_eta) return fail(DCM_E_INVALID, "NULL argument");
    if (!std::isfinite(h_xi_eta[0]) || !std::isfinite(h_xi_eta[1]))
        return fail(DCM_E_INVALID, "thermostat state must be finite");
    hipStream_t st = (hipStream_t)stream;
    const double t[2] = {h_xi_eta[0], h_xi_eta[1]};
    (void)hipMemcpyAsync(s->nh, t, sizeof t, hipMemcpyHostToDevice, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(DCM_E_HIP, "dcm_set_thermostat: %s", hipGetErrorString(e));
    return hip_status("dcm_set_thermostat");
}

dcm_status dcm_get_state(dcm_system *s, dcm_stream_t stream, double *d_x, double *d_v, double *d_rc,
                         int64_t *h_step)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    hipStream_t st = (hipStream_t)stream;
    if (d_x || d_v || d_rc)
        launch_unsort(s->set[s->cur], s->fx, s->fy, s->fz, s->n, d_x, d_v, d_rc, nullptr, st);
    if (h_step) *h_step = s->k;
    return hip_status("dcm_get_state");
}

dcm_status dcm_check(dcm_system *s, dcm_stream_t stream)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    hipStream_t st = (hipStream_t)stream;
    uint32_t flags = 0;
    (void)hipMemcpyAsync(&flags, s->gw.flags, sizeof flags, hipMemcpyDeviceToHost, st);
    hipError_t e = hipStreamSynchronize(st);
    if (e != hipSuccess) return fail(DCM_E_HIP, "dcm_check: %s", hipGetErrorString(e));
    if (flags & kFlagNonFinite) return fail(DCM_E_NONFINITE, "non-finite forces were produced");
    if (flags & kFlagNotConverged) return fail(DCM_E_NOT_CONVERGED, "distance sweeps hit their limit");
    if (flags & kFlagHistOverflow) return fail(DCM_E_INVALID, "smoothed counts exceed the histogram range");
    if (flags & kFlagBadCutoff) return fail(DCM_E_INVALID, "a cutoff lies outside [rc_min, rc_max]");
    if (flags & kFlagListOverflow) return fail(DCM_E_INVALID, "a neighbour list exceeded list_capacity");
    return DCM_OK;
}

dcm_status dcm_set_profiling(dcm_system *s, int32_t on)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    if (on < 0 || on > 2) return fail(DCM_E_INVALID, "profiling level must be 0, 1 or 2");
    s->profiling = on;
    return DCM_OK;
}

dcm_status dcm_stage_times(dcm_system *s, double *h_ms, int64_t *h_counts)
{
    if (!s) return fail(DCM_E_INVALID, "system is NULL");
    for (Event &e : s->events) {
        if (hipEventSynchronize(e.b) != hipSuccess) return fail(DCM_E_HIP, "event synchronize failed");
        float t = 0.f;
        (void)hipEventElapsedTime(&t, e.a, e.b);
        s->ms[e.stage] += t;
        s->counts[e.stage] += 1;
        s->spare.push_back(e);
    }
    s->events.clear();
    for (int q = 0; q < DCM_NSTAGES; ++q) {
        if (h_ms) h_ms[q] = s->ms[q];
        if (h_counts) h_counts[q] = s->counts[q];
    }
    return DCM_OK;
}

dcm_status dcm_list_builds(dcm_system *s, int64_t *h_builds)
{
    if (!s || !h_builds) return fail(DCM_E_INVALID, "NULL argument");
    *h_builds = s->list_builds;
    return DCM_OK;
}

dcm_status dcm_destroy(dcm_system *s)
{
    if (!s) return DCM_OK;
    for (Event &e : s->events) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    for (Event &e : s->spare) { (void)hipEventDestroy(e.a); (void)hipEventDestroy(e.b); }
    delete s;
    return DCM_OK;
}

// ---- grid stages on caller images ----------------------------------------------------
static size_t grid_layout(const Grid &g, GridWork &w, void *ws, double cap)
{
    Bump b(ws);
    const int64_t G = g.G;
    w.cell_start = nullptr;
    w.g = b.take<uint32_t>(G);
    w.gtmp = b.take<uint32_t>(G);
    w.raw = b.take<uint8_t>(G);
    w.label = b.take<uint8_t>(G);
    w.parent = b.take<uint32_t>(G);
    w.csize = b.take<uint32_t>(G);
    w.dist = nullptr;
    w.hist = b.take<uint32_t>(kHistBins);
    w.km = b.take<double>(3);
    w.stats = b.take<long long>(8);
    w.changed = b.take<uint32_t>(max_distance_sweeps(g, cap) + 1);
    w.flags = b.take<uint32_t>(1);
    w.tdirty = b.take<uint32_t>(2 * distance_tiles(g));
    w.tcur = b.take<uint32_t>(2 * distance_tiles(g));
    w.dist2 = b.take<double>(G);
    w.ctile = b.take<uint8_t>(component_tiles(g));
    w.dist_v = nullptr;
    w.ms = MsWork{nullptr, nullptr, nullptr, nullptr};
    return b.off + 256;
}

static dcm_status grid_from_dims(const int32_t dims[3], Grid &g)
{
    if (!dims) return fail(DCM_E_INVALID, "dims is NULL");
    for (int k = 0; k < 3; ++k) {
        if (dims[k] < 3) return fail(DCM_E_INVALID, "every grid dimension must be >= 3");
        g.n[k] = dims[k];
        g.h[k] = 1.0;
        g.L[k] = dims[k];
    }
    g.G = (int64_t)dims[0] * dims[1] * dims[2];
    g.sx = g.sy = g.sz = 0;
    if (g.G >= ((int64_t)1 << 31)) return fail(DCM_E_INVALID, "grid too large");
    return DCM_OK;
}

static dcm_status grid_ws(const int32_t dims[3], void *d_ws, size_t ws_bytes, Grid &g, GridWork &w,
                          double cap)
{
    dcm_status rs = grid_from_dims(dims, g);
    if (rs != DCM_OK) return rs;
    size_t need = grid_layout(g, w, nullptr, cap);
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < need)
        return fail(DCM_E_WORKSPACE, "grid workspace needs %zu bytes, 256-byte aligned", need);
    grid_layout(g, w, d_ws, cap);
    return DCM_OK;
}

// The sweep-counter array is sized for caps up to 64 boxes deep.
static const double kGridCapBound = 64.0;

dcm_status dcm_grid_workspace_bytes(const int32_t dims[3], size_t *bytes)
{
    Grid g;
    GridWork w;
    if (!bytes) return fail(DCM_E_INVALID, "bytes is NULL");
    dcm_status rs = grid_from_dims(dims, g);
    if (rs != DCM_OK) return rs;
    *bytes = grid_layout(g, w, nullptr, kGridCapBound);
    return DCM_OK;
}

dcm_status dcm_grid_smooth(const int32_t dims[3], int32_t passes, const uint32_t *d_in, uint32_t *d_out,
                           void *d_ws, size_t ws_bytes, dcm_stream_t stream)
{
    Grid g;
    GridWork w;
    dcm_status rs = grid_ws(dims, d_ws, ws_bytes, g, w, kGridCapBound);
    if (rs != DCM_OK) return rs;
    if (passes < 0 || passes > 4) return fail(DCM_E_INVALID, "passes must be 0..4");
    if (!d_in || !d_out) return fail(DCM_E_INVALID, "NULL image");
    launch_smooth(g, passes, nullptr, d_in, d_out, w.gtmp, (hipStream_t)stream);
    return hip_status("dcm_grid_smooth");
}

dcm_status dcm_grid_two_means(const int32_t dims[3], const uint32_t *d_g, double *d_km, int64_t *d_stats,
                              void *d_ws, size_t ws_bytes, dcm_stream_t stream)
{
    Grid g;
    GridWork w;
    dcm_status rs = grid_ws(dims, d_ws, ws_bytes, g, w, kGridCapBound);
    if (rs != DCM_OK) return rs;
    if (!d_g || !d_km) return fail(DCM_E_INVALID, "NULL argument");
    hipStream_t st = (hipStream_t)stream;
    launch_fill_u32(w.flags, 0u, 1, st);
    w.km = d_km;
    launch_two_means(g, d_g, w, (long long *)d_stats, false, st);
    return hip_status("dcm_grid_two_means");
}

dcm_status dcm_grid_segment(const int32_t dims[3], const uint32_t *d_g, const double *d_km,
                            int32_t min_component, uint8_t *d_raw, uint8_t *d_label, int64_t *d_stats,
                            void *d_ws, size_t ws_bytes, dcm_stream_t stream)
{
    Grid g;
    GridWork w;
    dcm_status rs = grid_ws(dims, d_ws, ws_bytes, g, w, kGridCapBound);
    if (rs != DCM_OK) return rs;
    if (!d_g || !d_km || !d_raw || !d_label) return fail(DCM_E_INVALID, "NULL argument");
    if (min_component < 0) return fail(DCM_E_INVALID, "min_component must be >= 0");
    hipStream_t st = (hipStream_t)stream;
    w.raw = d_raw;
    w.label = d_label;
    launch_fill_u32((uint32_t *)w.stats, 0u, 16, st);
    launch_segment(g, d_g, d_km, min_component, MsParams{0.0, 1.0, 0}, w, st);
    if (d_stats) launch_copy_bytes(d_stats, w.stats + 1, 4 * sizeof(long long), st);
    return hip_status("dcm_grid_segment");
}

dcm_status dcm_grid_distance(const int32_t dims[3], const double h[3], double cap, const uint8_t *d_label,
                             double *d_dist, int64_t *d_sweeps, void *d_ws, size_t ws_bytes,
                             dcm_stream_t stream)
{
    Grid g;
    GridWork w;
    dcm_status rs = grid_from_dims(dims, g);
    if (rs != DCM_OK) return rs;
    if (!h || !d_label || !d_dist) return fail(DCM_E_INVALID, "NULL argument");
    for (int k = 0; k < 3; ++k) {
        if (!(h[k] > 0.0)) return fail(DCM_E_INVALID, "box edges must be positive");
        g.h[k] = h[k];
        g.L[k] = h[k] * dims[k];
    }
    double hmin = std::min(h[0], std::min(h[1], h[2]));
    if (!(cap > 0.0) || cap / hmin > kGridCapBound) return fail(DCM_E_INVALID, "cap must be in (0, 64 h]");
    size_t need = grid_layout(g, w, nullptr, kGridCapBound * hmin);
    if (!d_ws || ((uintptr_t)d_ws & 255) || ws_bytes < need)
        return fail(DCM_E_WORKSPACE, "grid workspace needs %zu bytes, 256-byte aligned", need);
    grid_layout(g, w, d_ws, kGridCapBound * hmin);
    hipStream_t st = (hipStream_t)stream;
    launch_fill_u32(w.flags, 0u, 1, st);
    launch_fill_u32((uint32_t *)w.stats, 0u, 16, st);
    launch_distance(g, cap, d_label, kLabelVapor, d_dist, w, w.stats + 5, false, st);
    launch_cap_copy(d_dist, cap, d_dist, g.G, st);
    if (d_sweeps) launch_copy_bytes(d_sweeps, w.stats + 5, sizeof(long long), st);
    return hip_status("dcm_grid_distance");
}

}  // extern "C"
