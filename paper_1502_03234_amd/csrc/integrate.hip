// integrate.hip -- velocity-Verlet integration of Eq. 1-2 and the fixed-order reductions.
//
// A step is: v += dt/(2m) F, x += dt v, periodic wrap, re-binning, (detection), forces,
// v += dt/(2m) F. The closing half-kick of one step and the opening half-kick and drift of the
// next read the same forces, so inside a multi-step call they run as one streaming kernel
// (the kinetic energy of the completed step is taken between the two kicks); the arithmetic is
// the same sequence of operations as two separate kernels. Thermodynamic sums are formed per
// workgroup and then over workgroups in a fixed order, so every run gives the same bits.
//
// Under the Nose-Hoover thermostat a step is wrapped in two half thermostat steps (a symmetric
// Trotter splitting of the equations of motion with friction xi). The thermostat variables
// live on the device: the last wave of the thermo reduction, which owns the kinetic energy,
// advances them, and the streaming kernels read the velocity scale from device memory, so a
// thermostatted step needs no host round trip either.
#include "internal.h"
#include "launch.h"

namespace dcm {

namespace {

inline unsigned grid1(int64_t n) { return (unsigned)((n + kBlock - 1) / kBlock); }

__device__ double block_sum(double v)
{
    __shared__ double lds[kBlock / 64];
    for (int off = 32; off > 0; off >>= 1) v += __shfl_xor(v, off, 64);
    if ((threadIdx.x & 63) == 0) lds[threadIdx.x >> 6] = v;
    __syncthreads();
    double s = 0.0;
    for (int q = 0; q < kBlock / 64; ++q) s += lds[q];
    return s;
}

struct KFillU32 {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { uint32_t *p; uint32_t v; int64_t count; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        if (i < a.count) a.p[i] = a.v;
    }
};

struct KCopyBytes {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { uint8_t *dst; const uint8_t *src; size_t bytes; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        size_t i = ((size_t)blk * kThreads + threadIdx.x) * 16;
        if (i + 16 <= a.bytes && (((uintptr_t)a.dst | (uintptr_t)a.src) & 15) == 0) {
            *(uint4 *)(a.dst + i) = *(const uint4 *)(a.src + i);
        } else {
            for (size_t q = i; q < i + 16 && q < a.bytes; ++q) a.dst[q] = a.src[q];
        }
    }
};

struct KKickDriftKey {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        Grid g;
        PSet s;
        const double *fx, *fy, *fz;
        int64_t n;
        double hdt, dt;
        int second_kick;
        const double *scale;
        uint32_t *key;
        CellCounts counts;      // counts.cnt == nullptr: the keys are not counted here
        Partial *ke_partials;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KKickDriftKey::run(const Args &a, uint32_t blk, uint32_t)
{
    const Grid &g = a.g;
    const PSet &s = a.s;
    const double *fx = a.fx, *fy = a.fy, *fz = a.fz;
    const int64_t n = a.n;
    const double hdt = a.hdt, dt = a.dt;
    const int second_kick = a.second_kick;
    const double *scale = a.scale;
    int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    double ke = 0.0;
    uint32_t key = 0u;
    if (i < n) {
        double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
        const double f0 = fx[i], f1 = fy[i], f2 = fz[i];
        if (scale) {                  // opening thermostat half step
            const double c = *scale;
            vx = vx * c;
            vy = vy * c;
            vz = vz * c;
        }
        if (second_kick) {            // close the previous step
            vx = vx + hdt * f0;
            vy = vy + hdt * f1;
            vz = vz + hdt * f2;
            ke = vx * vx + vy * vy + vz * vz;
        }
        vx = vx + hdt * f0;
        vy = vy + hdt * f1;
        vz = vz + hdt * f2;
        double4 p = s.pos[i];
        p.x = wrap_periodic(p.x + dt * vx, g.L[0]);
        p.y = wrap_periodic(p.y + dt * vy, g.L[1]);
        p.z = wrap_periodic(p.z + dt * vz, g.L[2]);
        s.pos[i] = p;
        s.vx[i] = vx;
        s.vy[i] = vy;
        s.vz[i] = vz;
        key = pos_key(g, p.x, p.y, p.z);
        a.key[i] = key;
    }
    if (a.counts.cnt) {
        // the counting sort's count step, on the keys just computed
        const bool valid[1] = {i < n};
        const uint32_t k[1] = {key};
        const int64_t idx[1] = {i};
        count_cells<1>(valid, k, idx, a.counts.cnt, a.counts.rank, a.counts.bsum);
    }
    if (second_kick) {
        double t = block_sum(ke);
        if (threadIdx.x == 0) a.ke_partials[blk].ke = t;
    }
}

// mode 0: kinetic-energy partials only; 1: half kick v += hdt F; 2: thermostat scaling
// v *= *scale. Every mode leaves the workgroup's sum of |v|^2 (after the update) in ke_partials.
struct KKick {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        PSet s;
        const double *fx, *fy, *fz;
        int64_t n;
        double hdt;
        int mode;
        const double *scale;
        Partial *ke_partials;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KKick::run(const Args &a, uint32_t blk, uint32_t)
{
    const PSet &s = a.s;
    const double *fx = a.fx, *fy = a.fy, *fz = a.fz;
    const int64_t n = a.n;
    const double hdt = a.hdt;
    const int mode = a.mode;
    const double *scale = a.scale;
    int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    double ke = 0.0;
    if (i < n) {
        double vx = s.vx[i], vy = s.vy[i], vz = s.vz[i];
        if (mode == 1) {
            vx = vx + hdt * fx[i];
            vy = vy + hdt * fy[i];
            vz = vz + hdt * fz[i];
        } else if (mode == 2) {
            const double c = *scale;
            vx = vx * c;
            vy = vy * c;
            vz = vz * c;
        }
        if (mode != 0) {
            s.vx[i] = vx;
            s.vy[i] = vy;
            s.vz[i] = vz;
        }
        ke = vx * vx + vy * vy + vz * vz;
    }
    double t = block_sum(ke);
    if (threadIdx.x == 0) a.ke_partials[blk].ke = t;
}


// First stage of the thermo reduction: workgroup b sums its contiguous share of the force and
// kinetic-energy partials in a fixed order.
constexpr int kRedStage = 32;                      // workgroups of the first stage

struct KReduceStage {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { const Partial *fp; int nf; const Partial *kp; int nk; Partial *out_f, *out_k; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KReduceStage::run(const Args &a, uint32_t blk, uint32_t)
{
    const Partial *fp = a.fp, *kp = a.kp;
    const int nf = a.nf, nk = a.nk;
    __shared__ double lds[kBlock / 64][8];
    __shared__ long long ldp[kBlock / 64];
    const int fchunk = (nf + kRedStage - 1) / kRedStage, kchunk = (nk + kRedStage - 1) / kRedStage;
    const int f0 = (int)blk * fchunk, f1 = min(nf, f0 + fchunk);
    const int k0 = (int)blk * kchunk, k1 = min(nk, k0 + kchunk);
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long pc = 0;
    for (int q = f0 + threadIdx.x; q < f1; q += kBlock) {
        v[0] += fp[q].e;
        for (int r = 0; r < 6; ++r) v[1 + r] += fp[q].w[r];
        pc += fp[q].pairs;
    }
    for (int q = k0 + threadIdx.x; q < k1; q += kBlock) v[7] += kp[q].ke;
#pragma unroll
    for (int r = 0; r < 8; ++r)
        for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
    const int w = threadIdx.x >> 6;
    if ((threadIdx.x & 63) == 0) {
        for (int r = 0; r < 8; ++r) lds[w][r] = v[r];
        ldp[w] = pc;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        Partial pf = {}, pk = {};
        for (int q = 0; q < kBlock / 64; ++q) {
            pf.e += lds[q][0];
            for (int r = 0; r < 6; ++r) pf.w[r] += lds[q][1 + r];
            pf.pairs += ldp[q];
            pk.ke += lds[q][7];
        }
        a.out_f[blk] = pf;
        a.out_k[blk] = pk;
    }
}

// Half a Nose-Hoover step at kinetic energy K, on nh = {xi, eta, scale}: the friction advances
// a quarter step with G = (2K - g T*)/Q, the velocities (through the scale, and K with them)
// are damped by exp(-xi dt/2), eta advances half a step, and the friction its second quarter
// with the damped K. Returns the damped K.
__device__ double nh_half(double K, double *nh, const NhConst &c)
{
    double xi = nh[0], eta = nh[1];
    xi = xi + 0.25 * c.dt * ((2.0 * K - c.gT) / c.Q);
    const double sc = exp(-0.5 * c.dt * xi);
    K = K * sc * sc;
    eta = eta + 0.5 * c.dt * xi;
    xi = xi + 0.25 * c.dt * ((2.0 * K - c.gT) / c.Q);
    nh[0] = xi;
    nh[1] = eta;
    nh[2] = sc;
    return K;
}

// Second stage: one wave sums the first stage's results in a fixed order. nh_mode 0 writes the
// record (with the thermostat state nh, if given); kNhStart/kNhEnd also take half a thermostat
// step with the summed kinetic energy, kNhEnd recording the damped kinetic energy.
struct KReduceThermo {
    static constexpr int kThreads = 64, kWaves = 0;
    struct Args {
        const Partial *sf, *sk;
        double mass;
        long long step;
        dcm_thermo *out;
        double *nh;
        int nh_mode;
        NhConst c;
    };
    static __device__ void run(const Args &a, uint32_t, uint32_t);
};

__device__ void KReduceThermo::run(const Args &a, uint32_t, uint32_t)
{
    const Partial *sf = a.sf, *sk = a.sk;
    const double mass = a.mass;
    const long long step = a.step;
    dcm_thermo *out = a.out;
    double *nh = a.nh;
    const int nh_mode = a.nh_mode;
    const NhConst &c = a.c;
    const int q = threadIdx.x;
    double v[8] = {0, 0, 0, 0, 0, 0, 0, 0};
    long long pc = 0;
    if (q < kRedStage) {
        v[0] = sf[q].e;
        for (int r = 0; r < 6; ++r) v[1 + r] = sf[q].w[r];
        pc = sf[q].pairs;
        v[7] = sk[q].ke;
    }
#pragma unroll
    for (int r = 0; r < 8; ++r)
        for (int off = 32; off > 0; off >>= 1) v[r] += __shfl_xor(v[r], off, 64);
    for (int off = 32; off > 0; off >>= 1) pc += __shfl_xor(pc, off, 64);
    if (q == 0) {
        double ke = 0.5 * mass * v[7];
        if (nh_mode != kNhNone) ke = nh_half(ke, nh, c);
        if (out) {
            dcm_thermo t = {};
            t.pe = v[0];
            for (int r = 0; r < 6; ++r) t.virial[r] = v[1 + r];
            t.pairs = pc;
            t.ke = ke;
            t.step = step;
            t.xi = nh ? nh[0] : 0.0;
            t.eta = nh ? nh[1] : 0.0;
            *out = t;
        }
    }
}

struct KUnsort {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args {
        PSet s;
        const double *fx, *fy, *fz;
        int64_t n;
        double *x_out, *v_out, *rc_out, *f_out;
    };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KUnsort::run(const Args &a, uint32_t blk, uint32_t)
{
    const PSet &s = a.s;
    const double *fx = a.fx, *fy = a.fy, *fz = a.fz;
    const int64_t n = a.n;
    double *x_out = a.x_out, *v_out = a.v_out, *rc_out = a.rc_out, *f_out = a.f_out;
    int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    if (i >= n) return;
    const uint32_t id = s.id[i];
    if (x_out || rc_out) {
        double4 p = s.pos[i];
        if (x_out) { x_out[id] = p.x; x_out[n + id] = p.y; x_out[2 * n + id] = p.z; }
        if (rc_out) rc_out[id] = p.w;
    }
    if (v_out) { v_out[id] = s.vx[i]; v_out[n + id] = s.vy[i]; v_out[2 * n + id] = s.vz[i]; }
    if (f_out) { f_out[id] = fx[i]; f_out[n + id] = fy[i]; f_out[2 * n + id] = fz[i]; }
}

struct KLoadState {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { PSet s; const double *x, *v, *rc; int64_t n; double rc_fill; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t);
};

__device__ void KLoadState::run(const Args &a, uint32_t blk, uint32_t)
{
    const PSet &s = a.s;
    const double *x = a.x, *v = a.v, *rc = a.rc;
    const int64_t n = a.n;
    const double rc_fill = a.rc_fill;
    int64_t i = (int64_t)blk * kThreads + threadIdx.x;
    if (i >= n) return;
    s.pos[i] = make_double4(x[i], x[n + i], x[2 * n + i], rc ? rc[i] : rc_fill);
    s.vx[i] = v[i];
    s.vy[i] = v[n + i];
    s.vz[i] = v[2 * n + i];
    s.id[i] = (uint32_t)i;
}

struct KScatterRc {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { PSet s; const double *rc_in; int64_t n; double rc_min, rc_max; uint32_t *flags; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        if (i >= a.n) return;
        double r = a.rc_in[a.s.id[i]];
        if (!(r >= a.rc_min && r <= a.rc_max)) atomicOr(a.flags, kFlagBadCutoff);
        a.s.pos[i].w = r;
    }
};

struct KCheckFinite {
    static constexpr int kThreads = kBlock, kWaves = 0;
    struct Args { const double *v; int64_t count; uint32_t *flags; };
    static __device__ void run(const Args &a, uint32_t blk, uint32_t)
    {
        int64_t i = (int64_t)blk * kThreads + threadIdx.x;
        bool bad = i < a.count && !isfinite(a.v[i]);
        if (__ballot(bad) && __lane_id() == 0) atomicOr(a.flags, kFlagNonFinite);
    }
};

}  // namespace

int stream_blocks(int64_t n) { return (int)grid1(n); }

void launch_fill_u32(uint32_t *p, uint32_t v, int64_t count, hipStream_t st)
{
    if (count <= 0) return;
    emit<KFillU32>({p, v, count}, grid1(count), st);
}

void launch_copy_bytes(void *dst, const void *src, size_t bytes, hipStream_t st)
{
    if (bytes == 0) return;
    size_t chunks = (bytes + 15) / 16;
    emit<KCopyBytes>({(uint8_t *)dst, (const uint8_t *)src, bytes}, grid1((int64_t)chunks), st);
}

void launch_kick_drift_key(const Grid &g, PSet s, const double *fx, const double *fy,
                           const double *fz, int64_t n, double hdt, double dt, int second_kick,
                           const double *scale, uint32_t *key, CellCounts counts, Partial *ke_partials,
                           hipStream_t st)
{
    emit<KKickDriftKey>({g, s, fx, fy, fz, n, hdt, dt, second_kick, scale, key, counts, ke_partials}, grid1(n), st);
}

void launch_kick(PSet s, const double *fx, const double *fy, const double *fz, int64_t n,
                 double hdt, Partial *ke_partials, hipStream_t st)
{
    emit<KKick>({s, fx, fy, fz, n, hdt, 1, nullptr, ke_partials}, grid1(n), st);
}

void launch_scale(PSet s, int64_t n, const double *scale, Partial *ke_partials, hipStream_t st)
{
    emit<KKick>({s, nullptr, nullptr, nullptr, n, 0.0, 2, scale, ke_partials}, grid1(n), st);
}

void launch_ke_only(PSet s, int64_t n, Partial *ke_partials, hipStream_t st)
{
    emit<KKick>({s, nullptr, nullptr, nullptr, n, 0.0, 0, nullptr, ke_partials}, grid1(n), st);
}

void launch_reduce_thermo(const Partial *force_parts, int nforce, const Partial *ke_parts, int nke,
                          double mass, long long step, dcm_thermo *out, Partial *stage, double *nh,
                          int nh_mode, const NhConst &c, hipStream_t st)
{
    emit<KReduceStage>({force_parts, nforce, ke_parts, nke, stage, stage + kRedStage}, kRedStage, st);
    emit<KReduceThermo>({stage, stage + kRedStage, mass, step, out, nh, nh_mode, c}, 1, st);
}

int reduce_stage_partials() { return 2 * kRedStage; }

void launch_unsort(PSet s, const double *fx, const double *fy, const double *fz, int64_t n,
                   double *x_out, double *v_out, double *rc_out, double *f_out, hipStream_t st)
{
    emit<KUnsort>({s, fx, fy, fz, n, x_out, v_out, rc_out, f_out}, grid1(n), st);
}

void launch_load_state(PSet s, const double *x, const double *v, const double *rc, int64_t n,
                       double rc_fill, hipStream_t st)
{
    emit<KLoadState>({s, x, v, rc, n, rc_fill}, grid1(n), st);
}

void launch_scatter_rc(PSet s, const double *rc_in, int64_t n, double rc_min, double rc_max,
                       uint32_t *flags, hipStream_t st)
{
    emit<KScatterRc>({s, rc_in, n, rc_min, rc_max, flags}, grid1(n), st);
}

void launch_check_finite(const double *a, int64_t count, uint32_t *flags, hipStream_t st)
{
    emit<KCheckFinite>({a, count, flags}, grid1(count), st);
}

}  // namespace dcm
