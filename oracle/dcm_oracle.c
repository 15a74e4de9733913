/* dcm_oracle.c -- TEST INFRASTRUCTURE, not product code.
 *
 * Plain single-threaded FP64 oracle of the dynamic cutoff method (DCM) hot path.
 * Each function follows one passage of the thesis in the order it is written there:
 *
 *   orc_wrap / orc_bin      Section 4, Eq. 9-10 (boxes of edge L/N, particle counts)
 *   orc_smooth              smoothing of the count image (stands in for the perimeter
 *                           penalty of Eq. 13; integer [1,2,1] per axis, periodic)
 *   orc_two_means           Section 4.1, Eq. 14 (K-means with K = 2 on the box values)
 *   orc_components /
 *   orc_segment             Eq. 11-12 labels; Section 4.2, Alg. 4.1 connected components
 *                           (here a breadth-first flood fill), small-component removal
 *   orc_mumford_shah /
 *   orc_ms_solve            Section 4.1, Eq. 13 (two-phase piecewise-constant Mumford-Shah
 *                           segmentation; convex relaxation solved by a primal-dual method)
 *   orc_distance            Section 4.3, Eq. 15-19, Alg. 4.2 (fast sweeping, repeated
 *                           until nothing changes; band limited as in Section 4.3.2)
 *   orc_interp              Section 3, Eq. 5-6, Alg. 3.1 (trilinear interpolation)
 *   orc_cutoff              Section 3.1, Eq. 7-8 (exponential cutoff function; or the
 *                           linear ramp that Section 6 compares it with; optionally applied
 *                           to vapor particles by their depth into the vapor, Section 3.1)
 *   orc_forces              Section 2.2, Eq. 4 and Section 3.2, Alg. 3.2 (full pair loop,
 *                           the pair is used iff r < r_c[i]; only f_i is updated)
 *   orc_forces_images       the exact forces of Eq. 20's accuracy measure: Eq. 4 with no
 *                           cutoff, over every periodic image within a radius R
 *   orc_tail_planar /
 *   orc_tail                the runtime tail correction of Section 7, Eq. 21-22: the pair
 *                           energy and force beyond r_c[i] for a planar liquid/vapor model
 *                           placed by a signed box distance (radial quadrature)
 *   orc_run                 Eq. 1-2 advanced with velocity Verlet; optionally at constant
 *                           temperature (the thesis's runs are NVT, Section 6) with one
 *                           Nose-Hoover thermostat in a symmetric splitting
 *
 * No blocking, fusion or reordering beyond what those passages state.
 * Build: gcc -O2 -ffp-contract=off (no fast-math).
 */
#include "dcm_oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>

#define IDX(d, i, j, k) ((int64_t)((k) * (int64_t)(d)[1] + (j)) * (d)[0] + (i))

static int64_t pmod(int64_t a, int64_t n) { int64_t r = a % n; return r < 0 ? r + n : r; }

/* ---- grid (Eq. 10): N_k = max(3, round(L_k / bin)), box edge h_k = L_k / N_k ---------- */
int orc_grid(const orc_params *p, int32_t dims[3], double h[3])
{
    for (int k = 0; k < 3; ++k) {
        int64_t nk = (int64_t)round(p->box[k] / p->bin);
        if (nk < 3) nk = 3;
        dims[k] = (int32_t)nk;
        h[k] = p->box[k] / (double)nk;
    }
    return 0;
}

/* ---- periodic wrap into [0, L) --------------------------------------------------------- */
/* x mod L. When |x| is so large that the remainder has no significant digits left, the result
 * can land outside [0, L) after rounding; it is then taken as 0, so every wrapped position lies
 * in the box. */
static double wrap1(double x, double L)
{
    double t = x - L * floor(x / L);
    if (t < 0.0) t += L;
    if (t < 0.0 || t >= L) t = 0.0;
    return t;
}

void orc_wrap(const orc_params *p, int64_t n, double *x)
{
    for (int k = 0; k < 3; ++k)
        for (int64_t i = 0; i < n; ++i) x[k * n + i] = wrap1(x[k * n + i], p->box[k]);
}

static int32_t box_of(double x, double h, int32_t N)
{
    int64_t i = (int64_t)floor(x / h);
    if (i > N - 1) i = N - 1;
    if (i < 0) i = 0;
    return (int32_t)i;
}

/* ---- binning (Eq. 9): b_ijk = number of particles inside box (i,j,k) ------------------- */
void orc_bin(const orc_params *p, int64_t n, const double *x, uint32_t *count, uint32_t *cell)
{
    int32_t d[3]; double h[3];
    orc_grid(p, d, h);
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    memset(count, 0, sizeof(uint32_t) * (size_t)G);
    for (int64_t i = 0; i < n; ++i) {
        int32_t a = box_of(x[i], h[0], d[0]);
        int32_t b = box_of(x[n + i], h[1], d[1]);
        int32_t c = box_of(x[2 * n + i], h[2], d[2]);
        int64_t id = IDX(d, a, b, c);
        count[id] += 1;
        if (cell) cell[i] = (uint32_t)id;
    }
}

/* ---- smoothing: `passes` times, periodic [1,2,1] along x, then y, then z ---------------- */
void orc_smooth(const int32_t d[3], int32_t passes, const uint32_t *in, uint32_t *out)
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    uint32_t *tmp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)G);
    memcpy(out, in, sizeof(uint32_t) * (size_t)G);
    for (int32_t ps = 0; ps < passes; ++ps) {
        for (int ax = 0; ax < 3; ++ax) {
            for (int32_t k = 0; k < d[2]; ++k)
                for (int32_t j = 0; j < d[1]; ++j)
                    for (int32_t i = 0; i < d[0]; ++i) {
                        int32_t lo[3] = {i, j, k}, hi[3] = {i, j, k};
                        lo[ax] = (int32_t)pmod((int64_t)lo[ax] - 1, d[ax]);
                        hi[ax] = (int32_t)pmod((int64_t)hi[ax] + 1, d[ax]);
                        tmp[IDX(d, i, j, k)] = out[IDX(d, lo[0], lo[1], lo[2])]
                                             + 2u * out[IDX(d, i, j, k)]
                                             + out[IDX(d, hi[0], hi[1], hi[2])];
                    }
            memcpy(out, tmp, sizeof(uint32_t) * (size_t)G);
        }
    }
    free(tmp);
}

/* ---- two-means (Eq. 14 with K = 2, Lloyd's iteration) ----------------------------------
 * Start from the naive estimates rho_v = min b, rho_l = max b (Section 4.1). A box goes to
 * the liquid cluster iff its value is above the midpoint of the two centres (ties: vapor),
 * each centre becomes the mean of its cluster (exact integer sums, one FP64 division),
 * until the assignment stops changing. km = {rho_v, rho_l, threshold}. A constant image
 * has no interface: every box is liquid (threshold below the constant). */
int32_t orc_two_means(int64_t G, const uint32_t *g, double km[3])
{
    uint32_t mn = g[0], mx = g[0];
    for (int64_t c = 1; c < G; ++c) { if (g[c] < mn) mn = g[c]; if (g[c] > mx) mx = g[c]; }
    if (mn == mx) { km[0] = mn; km[1] = mx; km[2] = (double)mn - 1.0; return 0; }
    double cv = (double)mn, cl = (double)mx;
    int64_t prev = -1;
    int32_t it;
    for (it = 1; it <= 1000; ++it) {
        double m = 0.5 * (cv + cl);
        int64_t sv = 0, nv = 0, sl = 0, nl = 0;
        for (int64_t c = 0; c < G; ++c) {
            if ((double)g[c] > m) { sl += g[c]; nl += 1; }
            else                  { sv += g[c]; nv += 1; }
        }
        cv = (double)sv / (double)nv;
        cl = (double)sl / (double)nl;
        if (nl == prev) break;
        prev = nl;
    }
    km[0] = cv; km[1] = cl; km[2] = 0.5 * (cv + cl);
    return it;
}

/* ---- connected components of one phase (Section 4.2) ---------------------------------
 * 6-connected with periodic wrap; breadth-first flood fill started from every unvisited
 * box in increasing linear order, so each component is named by its smallest linear
 * index. comp[c] = that name (UINT32_MAX for boxes of the other phase), size[c] = size of
 * c's component. Returns the number of components. */
int64_t orc_components(const int32_t d[3], const uint8_t *s, uint8_t phase, uint32_t *comp,
                       uint32_t *size)
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    int64_t *queue = (int64_t *)malloc(sizeof(int64_t) * (size_t)G);
    for (int64_t c = 0; c < G; ++c) comp[c] = UINT32_MAX;
    int64_t ncomp = 0;
    for (int64_t c0 = 0; c0 < G; ++c0) {
        if (s[c0] != phase || comp[c0] != UINT32_MAX) continue;
        int64_t head = 0, tail = 0;
        queue[tail++] = c0;
        comp[c0] = (uint32_t)c0;
        while (head < tail) {
            int64_t c = queue[head++];
            int64_t i = c % d[0], j = (c / d[0]) % d[1], k = c / ((int64_t)d[0] * d[1]);
            int64_t nb[6] = {
                IDX(d, pmod(i - 1, d[0]), j, k), IDX(d, pmod(i + 1, d[0]), j, k),
                IDX(d, i, pmod(j - 1, d[1]), k), IDX(d, i, pmod(j + 1, d[1]), k),
                IDX(d, i, j, pmod(k - 1, d[2])), IDX(d, i, j, pmod(k + 1, d[2]))};
            for (int q = 0; q < 6; ++q)
                if (s[nb[q]] == phase && comp[nb[q]] == UINT32_MAX) {
                    comp[nb[q]] = (uint32_t)c0;
                    queue[tail++] = nb[q];
                }
        }
        for (int64_t q = 0; q < tail; ++q) size[queue[q]] = (uint32_t)tail;
        ncomp += 1;
    }
    for (int64_t c = 0; c < G; ++c) if (comp[c] == UINT32_MAX) size[c] = 0;
    free(queue);
    return ncomp;
}

/* ---- labels (Eq. 11-12) and removal of small components (Section 4.2, Fig. 20) --------
 * s = 0 (liquid) iff g > t, else 1 (vapor). Vapor components with fewer than
 * min_component boxes become liquid; then, on the updated image, liquid components with
 * fewer than min_component boxes become vapor.
 * stats = {vapor comps removed, liquid comps removed, vapor boxes flipped, liquid flipped} */
static void remove_small(const int32_t d[3], int32_t min_component, uint8_t *label, int64_t stats[4]);

void orc_segment(const int32_t d[3], const uint32_t *g, double t, int32_t min_component,
                 uint8_t *raw, uint8_t *label, int64_t stats[4])
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    for (int64_t c = 0; c < G; ++c) { raw[c] = ((double)g[c] > t) ? 0 : 1; label[c] = raw[c]; }
    remove_small(d, min_component, label, stats);
}

/* Section 4.2: vapor components smaller than min_component boxes become liquid, then liquid
 * components smaller than that (on the updated labels) become vapor. */
static void remove_small(const int32_t d[3], int32_t min_component, uint8_t *label, int64_t stats[4])
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    uint32_t *comp = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)G);
    uint32_t *size = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)G);
    for (int pass = 0; pass < 2; ++pass) {
        uint8_t phase = pass == 0 ? 1 : 0;
        orc_components(d, label, phase, comp, size);
        int64_t comps = 0, boxes = 0;
        for (int64_t c = 0; c < G; ++c) {
            if (label[c] == phase && size[c] < (uint32_t)min_component) {
                if (comp[c] == (uint32_t)c) comps += 1;
                boxes += 1;
            }
        }
        for (int64_t c = 0; c < G; ++c)
            if (label[c] == phase && size[c] < (uint32_t)min_component) label[c] = (uint8_t)(1 - phase);
        stats[pass] = comps;
        stats[2 + pass] = boxes;
    }
    free(comp);
    free(size);
}

/* ---- two-phase piecewise-constant Mumford-Shah segmentation (Eq. 13) --------------------
 * Eq. 13 with its data terms in the intended pairing (the liquid set against rho_l, the vapor
 * set against rho_v; the print swaps them) and the two densities fixed at the two-means centres
 * (Section 4.1). The labelling is minimised through its convex relaxation: over u in [0, 1]^G
 * (u = 1 liquid),
 *     sum_c u_c r_c + sum_c sum_k w_k |u(c + e_k) - u(c)|,  r_c = (f_c - rho_l)^2 - (f_c - rho_v)^2,
 * whose perimeter term is the anisotropic total variation (faces of the box grid, periodic);
 * for it the coarea formula holds, so every level set {u > t}, 0 < t < 1, of a minimiser is a
 * minimising labelling (Chan, Esedoglu and Nikolova 2006). The minimiser is sought by the
 * primal-dual algorithm of Chambolle and Pock (2011, Algorithm 1, theta = 1) with steps
 * sigma = tau = 1 / sqrt(12) (the squared norm of the forward-difference operator is at most
 * 12): per iteration
 *     p_k <- clamp(p_k + sigma (ubar(c + e_k) - ubar(c)), -w_k, w_k)        (dual, per axis)
 *     u'  <- clamp(u - tau (r - div p), 0, 1),  div p = sum_k (p_k(c) - p_k(c - e_k))
 *     ubar <- 2 u' - u,  u <- u'
 * from u = ubar = the threshold labelling and p = 0, for a fixed number of iterations; then
 * liquid iff u > 1/2. The per-element operations are in the order written. */
void orc_ms_solve(const int32_t d[3], const double *r, const double w[3], int32_t iters, double *u)
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    double *ub = (double *)malloc(sizeof(double) * (size_t)G);
    double *p = (double *)calloc((size_t)G * 3, sizeof(double));
    const double sigma = 1.0 / sqrt(12.0), tau = sigma;
    memcpy(ub, u, sizeof(double) * (size_t)G);
    for (int32_t it = 0; it < iters; ++it) {
        for (int32_t k = 0; k < d[2]; ++k)
            for (int32_t j = 0; j < d[1]; ++j)
                for (int32_t i = 0; i < d[0]; ++i) {
                    int64_t c = IDX(d, i, j, k);
                    int64_t nb[3] = {IDX(d, pmod(i + 1, d[0]), j, k), IDX(d, i, pmod(j + 1, d[1]), k),
                                     IDX(d, i, j, pmod(k + 1, d[2]))};
                    for (int a = 0; a < 3; ++a) {
                        double v = p[a * G + c] + sigma * (ub[nb[a]] - ub[c]);
                        p[a * G + c] = fmin(fmax(v, -w[a]), w[a]);
                    }
                }
        for (int32_t k = 0; k < d[2]; ++k)
            for (int32_t j = 0; j < d[1]; ++j)
                for (int32_t i = 0; i < d[0]; ++i) {
                    int64_t c = IDX(d, i, j, k);
                    int64_t nb[3] = {IDX(d, pmod(i - 1, d[0]), j, k), IDX(d, i, pmod(j - 1, d[1]), k),
                                     IDX(d, i, j, pmod(k - 1, d[2]))};
                    double div = ((p[c] - p[nb[0]]) + (p[G + c] - p[G + nb[1]])) + (p[2 * G + c] - p[2 * G + nb[2]]);
                    double un = fmin(fmax(u[c] - tau * (r[c] - div), 0.0), 1.0);
                    ub[c] = 2.0 * un - u[c];
                    u[c] = un;
                }
    }
    free(ub);
    free(p);
}

/* Eq. 13 on the density image g (the image the two-means centres came from), in units where
 * the liquid centre is 1 and the longest box edge L_max is 1: f = g / rho_l, and per unit box
 * volume a face normal to axis k weighs nu L_max / h_k. raw holds the threshold labels on entry
 * and the minimiser's labels (0 liquid, 1 vapor) on exit; u (optional) the relaxed field. */
void orc_mumford_shah(const int32_t d[3], const double h[3], double Lmax, const uint32_t *g,
                      const double km[3], double nu, int32_t iters, uint8_t *raw, double *u_out)
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    if (!(km[1] > 0.0)) return;                       /* empty image: nothing to segment */
    double *r = (double *)calloc((size_t)G, sizeof(double));
    double *u = (double *)calloc((size_t)G, sizeof(double));
    double cv = km[0] / km[1];
    for (int64_t c = 0; c < G; ++c) {
        double f = (double)g[c] / km[1];
        double fl = f - 1.0, fv = f - cv;
        r[c] = fl * fl - fv * fv;
        u[c] = raw[c] == 0 ? 1.0 : 0.0;
    }
    double w[3] = {nu * Lmax / h[0], nu * Lmax / h[1], nu * Lmax / h[2]};
    orc_ms_solve(d, r, w, iters, u);
    for (int64_t c = 0; c < G; ++c) raw[c] = u[c] > 0.5 ? 0 : 1;
    if (u_out) memcpy(u_out, u, sizeof(double) * (size_t)G);
    free(r);
    free(u);
}

/* ---- Godunov upwind update (Eq. 16-18, three dimensions, per-axis spacing) -------------
 * a[k] = min of the two neighbours along axis k. Solve sum_k ((d - a_k)^+ / h_k)^2 = 1:
 * sort the a_k ascending (ties by axis), take d = a_1 + h_1, and while d exceeds the next
 * a_k include that axis and take the larger root of the quadratic. With w_k = 1/h_k^2 the
 * root is (sum w a + sqrt(sum w - sum_{k<l} w_k w_l (a_k - a_l)^2)) / sum w. */
double orc_godunov(const double a_in[3], const double h_in[3])
{
    double a[3] = {a_in[0], a_in[1], a_in[2]}, h[3] = {h_in[0], h_in[1], h_in[2]};
    for (int p = 0; p < 2; ++p)                      /* stable sort of three (a, h) pairs */
        for (int q = 0; q < 2 - p; ++q)
            if (a[q + 1] < a[q]) {
                double ta = a[q]; a[q] = a[q + 1]; a[q + 1] = ta;
                double th = h[q]; h[q] = h[q + 1]; h[q + 1] = th;
            }
    if (isinf(a[0])) return INFINITY;
    double d = a[0] + h[0];
    if (d > a[1]) {
        double w0 = 1.0 / (h[0] * h[0]), w1 = 1.0 / (h[1] * h[1]);
        double sw = w0 + w1;
        double swa = w0 * a[0] + w1 * a[1];
        double dd = a[0] - a[1];
        double disc = sw - w0 * w1 * (dd * dd);
        if (disc < 0.0) disc = 0.0;
        d = (swa + sqrt(disc)) / sw;
        if (d > a[2]) {
            double w2 = 1.0 / (h[2] * h[2]);
            sw = w0 + w1 + w2;
            swa = w0 * a[0] + w1 * a[1] + w2 * a[2];
            double d01 = a[0] - a[1], d02 = a[0] - a[2], d12 = a[1] - a[2];
            disc = sw - (w0 * w1 * (d01 * d01) + w0 * w2 * (d02 * d02) + w1 * w2 * (d12 * d12));
            if (disc < 0.0) disc = 0.0;
            d = (swa + sqrt(disc)) / sw;
        }
    }
    return d;
}

/* ---- distance to the interface (Eq. 15-19, Alg. 4.2, band of Section 4.3.2) ------------
 * Vapor boxes are the zero set, liquid boxes start at +infinity. Gauss-Seidel sweeps in
 * the 2^3 alternating directions apply d_new = min(d_old, d_bar) (Eq. 19), keeping only
 * values <= cap (the band r_c^max + h); rounds of 8 sweeps repeat until a round changes
 * nothing. Afterwards every value above cap (including infinity) is set to cap.
 * Returns the number of rounds. */
int64_t orc_distance(const int32_t d[3], const double h[3], double cap, const uint8_t *label,
                     double *D)
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    for (int64_t c = 0; c < G; ++c) D[c] = label[c] == 1 ? 0.0 : INFINITY;
    int64_t rounds = 0;
    for (;;) {
        int64_t changed = 0;
        for (int dir = 0; dir < 8; ++dir) {
            int sx = (dir & 1) ? -1 : 1, sy = (dir & 2) ? -1 : 1, sz = (dir & 4) ? -1 : 1;
            for (int32_t kk = 0; kk < d[2]; ++kk) {
                int32_t k = sz > 0 ? kk : d[2] - 1 - kk;
                for (int32_t jj = 0; jj < d[1]; ++jj) {
                    int32_t j = sy > 0 ? jj : d[1] - 1 - jj;
                    for (int32_t ii = 0; ii < d[0]; ++ii) {
                        int32_t i = sx > 0 ? ii : d[0] - 1 - ii;
                        int64_t c = IDX(d, i, j, k);
                        if (label[c] == 1) continue;
                        double a[3];
                        a[0] = fmin(D[IDX(d, pmod(i - 1, d[0]), j, k)], D[IDX(d, pmod(i + 1, d[0]), j, k)]);
                        a[1] = fmin(D[IDX(d, i, pmod(j - 1, d[1]), k)], D[IDX(d, i, pmod(j + 1, d[1]), k)]);
                        a[2] = fmin(D[IDX(d, i, j, pmod(k - 1, d[2]))], D[IDX(d, i, j, pmod(k + 1, d[2]))]);
                        double db = orc_godunov(a, h);
                        if (db <= cap && db < D[c]) { D[c] = db; changed += 1; }
                    }
                }
            }
        }
        rounds += 1;
        if (!changed) break;
    }
    for (int64_t c = 0; c < G; ++c) if (D[c] > cap) D[c] = cap;
    return rounds;
}

/* ---- cutoff function (Eq. 7-8; linear ramp as the alternative of Section 6) ------------- */
double orc_cutoff(const orc_params *p, double d)
{
    if (p->rc_min == p->rc_max) return p->rc_max;
    if (d <= 0.0) return p->rc_max;
    if (d >= p->rc_max) return p->rc_min;
    if (p->cutoff_shape == 1)                  /* linear ramp from r_c^max at d = 0 */
        return p->rc_max + (p->rc_min - p->rc_max) * (d / p->rc_max);
    double a = (p->rc_max - p->rc_min) / (exp2(p->alpha * p->rc_max) - 1.0);
    double b = p->rc_min - a;
    return a * exp2(p->alpha * (p->rc_max - d)) + b;
}

/* ---- trilinear interpolation of box-centre distances (Alg. 3.1, Fig. 10-11) ------------
 * Box values sit at box centres. The lower-left-front box of a point has index
 * floor(x/h - 1/2) (periodic); the weights are the fractional offsets from it. Interpolate
 * along x first, then y, then z; lerp(a, b, t) = a + t (b - a). */
static double lerp(double a, double b, double t) { return a + t * (b - a); }

double orc_interp(const int32_t d[3], const double h[3], const double *D, const double xp[3])
{
    int64_t i0[3], i1[3];
    double t[3];
    for (int k = 0; k < 3; ++k) {
        double u = xp[k] / h[k] - 0.5;
        double f = floor(u);
        t[k] = u - f;
        i0[k] = pmod((int64_t)f, d[k]);
        i1[k] = pmod(i0[k] + 1, d[k]);
    }
    double c00 = lerp(D[IDX(d, i0[0], i0[1], i0[2])], D[IDX(d, i1[0], i0[1], i0[2])], t[0]);
    double c10 = lerp(D[IDX(d, i0[0], i1[1], i0[2])], D[IDX(d, i1[0], i1[1], i0[2])], t[0]);
    double c01 = lerp(D[IDX(d, i0[0], i0[1], i1[2])], D[IDX(d, i1[0], i0[1], i1[2])], t[0]);
    double c11 = lerp(D[IDX(d, i0[0], i1[1], i1[2])], D[IDX(d, i1[0], i1[1], i1[2])], t[0]);
    double c0 = lerp(c00, c10, t[1]);
    double c1 = lerp(c01, c11, t[1]);
    return lerp(c0, c1, t[2]);
}

/* Depth of the distance band (Section 4.3.2): one box beyond r_c^max, where the cutoff
 * function has reached r_c^min. The tail correction sees the interface further, to 2 r_c^max
 * plus a box (the proximity of 2 r_c that Section 7 suggests for its integral): beyond, the
 * planar force is below a sixteenth of its value at r_c^max. */
static double band_limit(const orc_params *p, const double h[3])
{
    double hmax = fmax(h[0], fmax(h[1], h[2]));
    return (p->tail ? 2.0 * p->rc_max : p->rc_max) + hmax;
}

/* Distance of every box to the liquid (the same solve with the roles of the phases swapped):
 * liquid boxes are the zero set. Used by the tail correction to place vapor particles. */
static int64_t vapor_distance(const int32_t d[3], const double h[3], double cap, const uint8_t *label,
                              double *D)
{
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    uint8_t *flip = (uint8_t *)malloc((size_t)G);
    for (int64_t c = 0; c < G; ++c) flip[c] = label[c] == 1 ? 0 : 1;
    int64_t r = orc_distance(d, h, cap, flip, D);
    free(flip);
    return r;
}

/* ---- the interface detection of Fig. 14, one call ------------------------------------- */
int orc_detect(const orc_params *p, int64_t n, const double *x, orc_detect_out *o)
{
    int32_t d[3]; double h[3];
    orc_grid(p, d, h);
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    orc_bin(p, n, x, o->count, NULL);
    orc_smooth(d, p->smooth_passes, o->count, o->smooth);
    o->stats[0] = orc_two_means(G, o->smooth, o->km);
    if (p->ms_nu > 0.0) {
        /* Eq. 13 in place of the plain threshold, then the removal of Section 4.2 */
        for (int64_t c = 0; c < G; ++c) o->raw[c] = ((double)o->smooth[c] > o->km[2]) ? 0 : 1;
        double Lmax = fmax(p->box[0], fmax(p->box[1], p->box[2]));
        orc_mumford_shah(d, h, Lmax, o->smooth, o->km, p->ms_nu, p->ms_iters, o->raw, NULL);
        memcpy(o->label, o->raw, (size_t)G);
        remove_small(d, p->min_component, o->label, o->stats + 1);
    } else {
        orc_segment(d, o->smooth, o->km[2], p->min_component, o->raw, o->label, o->stats + 1);
    }
    double cap = band_limit(p, h);
    o->stats[5] = orc_distance(d, h, cap, o->label, o->dist);
    int vapor_side = (p->tail || p->vapor_cutoff) && o->dist_v;
    if (vapor_side) vapor_distance(d, h, cap, o->label, o->dist_v);
    for (int64_t i = 0; i < n; ++i) {
        double xp[3] = {x[i], x[n + i], x[2 * n + i]};
        o->d[i] = orc_interp(d, h, o->dist, xp);
        /* vapor particles too (Section 3.1's extension of Eq. 7 to the low-density phase): the
         * cutoff of the larger of the two interpolated depths, which mirrors Eq. 7 about the
         * midplane between the last liquid and the first vapor box centre */
        double depth = o->d[i];
        if (p->vapor_cutoff && vapor_side) depth = fmax(depth, orc_interp(d, h, o->dist_v, xp));
        o->rc[i] = orc_cutoff(p, depth);
    }
    return 0;
}

/* ---- Lennard-Jones pair term (Eq. 4) ----------------------------------------------------
 * Minimum image: x_j is moved to its periodic image nearest x_i, then dx = x_i - x_j.
 * r^2 = dx^2 + dy^2 + dz^2 is formed with fused multiply-adds. Used iff r^2 < r_c^2
 * (Alg. 3.2; strict). F_i += (f/r) dx with f/r = 24 eps (2 (s/r)^12 - (s/r)^6) / r^2,
 * e_i += V(r)/2 (minus V(r_c)/2 if shifted), W_i += dx (x) f / 2. */
typedef struct { double f[3], e, w[6]; int64_t pairs; } acc_t;

static double lj_v(const orc_params *p, double r2)
{
    double sr2 = p->sigma * p->sigma / r2;
    double sr6 = sr2 * sr2 * sr2;
    return 4.0 * p->epsilon * sr6 * (sr6 - 1.0);
}

static void pair_term(const orc_params *p, const double *x, int64_t n, int64_t i, int64_t j,
                      const double *rc, acc_t *a)
{
    double dx[3];
    for (int k = 0; k < 3; ++k) {
        double L = p->box[k];
        double xi = x[k * n + i], xj = x[k * n + j];
        double img = rint((xi - xj) / L);
        dx[k] = xi - (xj + img * L);
    }
    double rcp = rc[i];
    if (p->pair_rule == 1 && rc[j] > rcp) rcp = rc[j];
    double rc2 = rcp * rcp;
    double r2 = fma(dx[2], dx[2], fma(dx[1], dx[1], dx[0] * dx[0]));
    if (!(r2 < rc2)) return;
    double sr2 = p->sigma * p->sigma / r2;
    double sr6 = sr2 * sr2 * sr2;
    double fr = 24.0 * p->epsilon * sr6 * (2.0 * sr6 - 1.0) / r2;
    double fx = fr * dx[0], fy = fr * dx[1], fz = fr * dx[2];
    a->f[0] += fx; a->f[1] += fy; a->f[2] += fz;
    double v = 4.0 * p->epsilon * sr6 * (sr6 - 1.0);
    if (p->energy_shift) v -= lj_v(p, rc2);
    a->e += 0.5 * v;
    a->w[0] += 0.5 * dx[0] * fx;
    a->w[1] += 0.5 * dx[1] * fy;
    a->w[2] += 0.5 * dx[2] * fz;
    a->w[3] += 0.5 * dx[0] * fy;
    a->w[4] += 0.5 * dx[0] * fz;
    a->w[5] += 0.5 * dx[1] * fz;
    a->pairs += 1;
}

static void store(acc_t *a, int64_t slot, int64_t m, double *f, double *e, double *w, int64_t *pairs)
{
    for (int k = 0; k < 3; ++k) f[k * m + slot] = a->f[k];
    if (e) e[slot] = a->e;
    if (w) for (int k = 0; k < 6; ++k) w[k * m + slot] = a->w[k];
    if (pairs) pairs[slot] = a->pairs;
}

/* Forces on every particle (subset == NULL, outputs [3][n], [n], [6][n], [n]) or on the
 * listed particles (outputs sized m). method 0: all j (O(N^2)); method 1: link cells of
 * edge >= r_c^max with the 27-cell stencil (Section 2.2.1), falling back to method 0
 * when fewer than 3 cells fit along an axis. */
void orc_forces(const orc_params *p, int64_t n, const double *x, const double *rc,
                int64_t m, const int64_t *subset, int32_t method,
                double *f, double *e, double *w, int64_t *pairs)
{
    if (!subset) m = n;
    int64_t nc[3];
    double ch[3];
    int use_cells = method == 1;
    for (int k = 0; k < 3; ++k) {
        nc[k] = (int64_t)floor(p->box[k] / p->rc_max);
        if (nc[k] < 3) use_cells = 0;
        ch[k] = p->box[k] / (double)(nc[k] > 0 ? nc[k] : 1);
    }
    if (!use_cells) {
        for (int64_t s = 0; s < m; ++s) {
            int64_t i = subset ? subset[s] : s;
            acc_t a; memset(&a, 0, sizeof a);
            for (int64_t j = 0; j < n; ++j) if (j != i) pair_term(p, x, n, i, j, rc, &a);
            store(&a, s, m, f, e, w, pairs);
        }
        return;
    }
    int64_t C = nc[0] * nc[1] * nc[2];
    int64_t *head = (int64_t *)malloc(sizeof(int64_t) * (size_t)C);
    int64_t *next = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    int64_t *cid = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    for (int64_t c = 0; c < C; ++c) head[c] = -1;
    for (int64_t j = n - 1; j >= 0; --j) {
        int64_t q[3];
        for (int k = 0; k < 3; ++k) {
            q[k] = (int64_t)floor(x[k * n + j] / ch[k]);
            if (q[k] > nc[k] - 1) q[k] = nc[k] - 1;
            if (q[k] < 0) q[k] = 0;
        }
        int64_t c = (q[2] * nc[1] + q[1]) * nc[0] + q[0];
        cid[j] = c;
        next[j] = head[c];
        head[c] = j;
    }
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = subset ? subset[s] : s;
        int64_t c = cid[i];
        int64_t ci = c % nc[0], cj = (c / nc[0]) % nc[1], ck = c / (nc[0] * nc[1]);
        acc_t a; memset(&a, 0, sizeof a);
        for (int dz = -1; dz <= 1; ++dz)
            for (int dy = -1; dy <= 1; ++dy)
                for (int dx = -1; dx <= 1; ++dx) {
                    int64_t nb = (pmod(ck + dz, nc[2]) * nc[1] + pmod(cj + dy, nc[1])) * nc[0]
                               + pmod(ci + dx, nc[0]);
                    for (int64_t j = head[nb]; j >= 0; j = next[j])
                        if (j != i) pair_term(p, x, n, i, j, rc, &a);
                }
        store(&a, s, m, f, e, w, pairs);
    }
    free(head); free(next); free(cid);
}

/* ---- exact reference forces (F^exact of Eq. 20) ------------------------------------------
 * The full Lennard-Jones force of Eq. 4, with no cutoff function, summed over every particle j
 * and every periodic image x_j + (a L_x, b L_y, c L_z) closer than R to x_i; R may exceed half
 * the box. The lattice sum converges absolutely, so only its part beyond R is missing. Outputs
 * for the listed particles (subset NULL: all n): f [3][m], e [m] = 1/2 sum_j V(r_ij). */
void orc_forces_images(const orc_params *p, int64_t n, const double *x, double R, int64_t m,
                       const int64_t *subset, double *f, double *e)
{
    int64_t K[3];
    for (int k = 0; k < 3; ++k) K[k] = (int64_t)ceil(R / p->box[k]) + 1;
    for (int64_t s = 0; s < m; ++s) {
        int64_t i = subset ? subset[s] : s;
        double acc[3] = {0.0, 0.0, 0.0}, en = 0.0;
        for (int64_t j = 0; j < n; ++j)
            for (int64_t a = -K[0]; a <= K[0]; ++a)
                for (int64_t b = -K[1]; b <= K[1]; ++b)
                    for (int64_t c = -K[2]; c <= K[2]; ++c) {
                        if (j == i && a == 0 && b == 0 && c == 0) continue;
                        double d[3];
                        d[0] = x[i] - (x[j] + (double)a * p->box[0]);
                        d[1] = x[n + i] - (x[n + j] + (double)b * p->box[1]);
                        d[2] = x[2 * n + i] - (x[2 * n + j] + (double)c * p->box[2]);
                        double r2 = d[0] * d[0] + d[1] * d[1] + d[2] * d[2];
                        if (!(r2 < R * R)) continue;
                        double sr2 = p->sigma * p->sigma / r2;
                        double sr6 = sr2 * sr2 * sr2;
                        double fr = 24.0 * p->epsilon * sr6 * (2.0 * sr6 - 1.0) / r2;
                        for (int k = 0; k < 3; ++k) acc[k] += fr * d[k];
                        en += 4.0 * p->epsilon * sr6 * (sr6 - 1.0);
                    }
        for (int k = 0; k < 3; ++k) f[k * m + s] = acc[k];
        if (e) e[s] = 0.5 * en;
    }
}

/* ---- Nose-Hoover thermostat ---------------------------------------------------------------
 * Equations of motion at constant temperature: dv/dt = f/m - xi v, dxi/dt = (sum m v^2 -
 * g T*)/Q, deta/dt = xi, with g = 3n - 3 thermalised degrees of freedom (the friction scales
 * the total momentum, which therefore stays at its initial value) and Q = g T* tau^2. The
 * quantity K + U + Q xi^2/2 + g T* eta is conserved. Half a thermostat step (dt/2), taken at
 * the start and at the end of each velocity-Verlet step: xi advances a quarter step at the
 * current K; the velocities are damped by exp(-xi dt/2); eta advances half a step; xi advances
 * its second quarter step at the damped K. */
static double kinetic(const orc_params *p, int64_t n, const double *v)
{
    double s = 0.0;
    for (int64_t i = 0; i < 3 * n; ++i) s += v[i] * v[i];
    return 0.5 * p->mass * s;
}

static void nh_half_step(const orc_params *p, int64_t n, double *v, double nh[2])
{
    double g = 3.0 * (double)n - 3.0;
    double gT = g * p->temperature;
    double Q = gT * p->tdamp * p->tdamp;
    double K = kinetic(p, n, v);
    nh[0] += 0.25 * p->dt * (2.0 * K - gT) / Q;
    double s = exp(-0.5 * p->dt * nh[0]);
    for (int64_t i = 0; i < 3 * n; ++i) v[i] *= s;
    nh[1] += 0.5 * p->dt * nh[0];
    K = kinetic(p, n, v);
    nh[0] += 0.25 * p->dt * (2.0 * K - gT) / Q;
}

/* ---- runtime tail correction (Section 7, Eq. 21-22) ------------------------------------
 * Eq. 22 adds to particle i the pair energy its cutoff leaves out: the integral of V(r) over
 * the points beyond r_c[i], weighted by the liquid density where they lie in the liquid and by
 * the vapor density where they lie in the vapor. Its force is the same integral of the pair
 * force -dV/dx_i (Eq. 21 applied under the integral, over the same pairs beyond the cutoff).
 * Model of the phases around i: a plane at distance |delta| from i, the liquid on the side of
 * the unit normal m (delta > 0: i is in the liquid, < 0: in the vapor). On the shell of radius
 * r about i the liquid is the cap cos(theta) > c0 = -delta / r (clamped to [-1, 1], theta
 * measured from m): its area is 2 pi r^2 (1 - c0) and its first moment, the integral of
 * cos(theta) over it, pi r^2 (1 - c0^2). Hence
 *   du = rho_v int_{r_c}^inf 4 pi r^2 V dr + (rho_l - rho_v) int_{r_c}^inf area(r) V(r) dr
 *   F  = m (rho_l - rho_v) int_{r_c}^inf moment(r) dV/dr dr
 * (a uniform density exerts no net force). Shells with r <= |delta| lie wholly in one phase
 * (moment 0). Every integral over [a, inf) is taken in t = a / r on (0, 1], where each
 * integrand below is a polynomial in t of degree at most 11, by a 12-point Gauss-Legendre
 * rule, exact up to rounding. */

/* Gauss-Legendre nodes and weights on [0, 1]: Newton's method on the Legendre polynomial P_m,
 * evaluated by Bonnet's recursion (j P_j = (2j - 1) z P_{j-1} - (j - 1) P_{j-2}). */
static void gauss_legendre01(int m, double *t, double *w)
{
    const double pi = acos(-1.0);
    for (int i = 0; i < m; ++i) {
        double z = cos(pi * (i + 0.75) / (m + 0.5)), dp = 1.0;
        for (int it = 0; it < 100; ++it) {
            double p0 = 1.0, p1 = 0.0;
            for (int j = 1; j <= m; ++j) {
                double p2 = p1;
                p1 = p0;
                p0 = ((2.0 * j - 1.0) * z * p1 - (j - 1.0) * p2) / j;
            }
            dp = m * (z * p0 - p1) / (z * z - 1.0);
            double step = p0 / dp;
            z -= step;
            if (fabs(step) <= 1e-15) break;
        }
        t[i] = 0.5 * (1.0 - z);
        w[i] = 1.0 / ((1.0 - z * z) * dp * dp);
    }
}

static double lj_vr(const orc_params *p, double r)
{
    double s6 = pow(p->sigma / r, 6.0);
    return 4.0 * p->epsilon * (s6 * s6 - s6);
}

static double lj_dv(const orc_params *p, double r)
{
    double s6 = pow(p->sigma / r, 6.0);
    return 4.0 * p->epsilon * (-12.0 * s6 * s6 + 6.0 * s6) / r;
}

/* kind 0: 4 pi r^2 V (whole shell); 1: liquid cap area times V (r > |delta|);
 * 2: liquid cap moment times dV/dr (r > |delta|) */
static double tail_integrand(const orc_params *p, int kind, double r, double delta)
{
    const double pi = acos(-1.0);
    if (kind == 0) return 4.0 * pi * r * r * lj_vr(p, r);
    double c0 = -delta / r;
    if (kind == 1) return 2.0 * pi * r * r * (1.0 - c0) * lj_vr(p, r);
    return pi * r * r * (1.0 - c0 * c0) * lj_dv(p, r);
}

static double radial(const orc_params *p, double a, int kind, double delta)
{
    double t[12], w[12], s = 0.0;
    gauss_legendre01(12, t, w);
    for (int i = 0; i < 12; ++i) {
        double r = a / t[i];
        s += w[i] * tail_integrand(p, kind, r, delta) * (a / (t[i] * t[i]));
    }
    return s;
}

void orc_tail_planar(const orc_params *p, double rc, double delta, double rho_l, double rho_v,
                     double *f_normal, double *du)
{
    double ad = fabs(delta), a = fmax(rc, ad), drho = rho_l - rho_v;
    double whole = radial(p, rc, 0, 0.0);
    /* shells between r_c and |delta| lie wholly in the liquid (delta > 0) or the vapor */
    double inner = (delta > 0.0 && ad > rc) ? whole - radial(p, ad, 0, 0.0) : 0.0;
    *du = rho_v * whole + drho * (inner + radial(p, a, 1, delta));
    *f_normal = drho * radial(p, a, 2, delta);
}

/* The eight boxes around xp (Alg. 3.1's indexing) and the fractional offsets. */
static void interp_corners(const int32_t d[3], const double h[3], const double xp[3], int64_t idx[8],
                           double t[3])
{
    int64_t i0[3], i1[3];
    for (int k = 0; k < 3; ++k) {
        double u = xp[k] / h[k] - 0.5;
        double f = floor(u);
        t[k] = u - f;
        i0[k] = pmod((int64_t)f, d[k]);
        i1[k] = pmod(i0[k] + 1, d[k]);
    }
    for (int q = 0; q < 8; ++q)
        idx[q] = IDX(d, (q & 1) ? i1[0] : i0[0], (q & 2) ? i1[1] : i0[1], (q & 4) ? i1[2] : i0[2]);
}

/* Trilinear interpolation (Eq. 6) and the gradient of the interpolant. */
double orc_interp_grad(const int32_t d[3], const double h[3], const double *D, const double xp[3],
                       double grad[3])
{
    int64_t idx[8];
    double t[3], val = 0.0;
    interp_corners(d, h, xp, idx, t);
    grad[0] = grad[1] = grad[2] = 0.0;
    for (int q = 0; q < 8; ++q) {
        double wx = (q & 1) ? t[0] : 1.0 - t[0];
        double wy = (q & 2) ? t[1] : 1.0 - t[1];
        double wz = (q & 4) ? t[2] : 1.0 - t[2];
        double v = D[idx[q]];
        val += wx * wy * wz * v;
        grad[0] += ((q & 1) ? 1.0 : -1.0) * wy * wz * v / h[0];
        grad[1] += wx * ((q & 2) ? 1.0 : -1.0) * wz * v / h[1];
        grad[2] += wx * wy * ((q & 4) ? 1.0 : -1.0) * v / h[2];
    }
    return val;
}

/* Tail correction of every particle from one detection's two distance fields.
 * Signed box value: depth into the liquid less half a box edge (the interface is taken
 * midway between the last liquid and the first vapor box centre), and minus the depth into
 * the vapor less half a box edge on vapor boxes; half a box edge is the mean of h / 2.
 * delta is the interpolated signed value at x_i and m the gradient of the interpolant (a
 * distance field has a unit gradient; where the field flattens at the band limit the force
 * fades with it). Where all eight boxes around x_i lie at the band limit (the capped depth,
 * less a relative 1e-9 so that rounding in the distances cannot move the decision) the
 * particle is deep in its phase: du is the uniform value of that phase and F = 0.
 * Densities: the two-means centres (km[1] liquid, km[0] vapor) over the box volume, divided by
 * 64 per smoothing pass (each pass multiplies a uniform image by 4 along each axis).
 * Outputs: f [3][n] and du [n] (Eq. 22's du_i; the pair-energy share of i is du_i / 2). */
void orc_tail(const orc_params *p, const double *Dl, const double *Dv, const double km[3], int64_t n,
              const double *x, const double *rc, double *f, double *du)
{
    int32_t d[3]; double h[3];
    orc_grid(p, d, h);
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    double cap = band_limit(p, h), s = (h[0] + h[1] + h[2]) / 6.0;
    double *phi = (double *)malloc(sizeof(double) * (size_t)G);
    for (int64_t c = 0; c < G; ++c) phi[c] = Dl[c] > 0.0 ? Dl[c] - s : -(Dv[c] - s);
    double norm = pow(64.0, p->smooth_passes) * h[0] * h[1] * h[2];
    double rho_v = km[0] / norm, rho_l = km[1] / norm;
    for (int64_t i = 0; i < n; ++i) {
        double xp[3] = {x[i], x[n + i], x[2 * n + i]};
        int64_t idx[8];
        double t[3], g[3];
        interp_corners(d, h, xp, idx, t);
        int deep = 1;
        for (int q = 0; q < 8; ++q) if (fabs(phi[idx[q]]) < (cap - s) * (1.0 - 1e-9)) deep = 0;
        f[i] = f[n + i] = f[2 * n + i] = 0.0;
        if (deep) {
            double rho = phi[idx[0]] > 0.0 ? rho_l : rho_v;
            du[i] = rho * radial(p, rc[i], 0, 0.0);
            continue;
        }
        double delta = orc_interp_grad(d, h, phi, xp, g), fn;
        orc_tail_planar(p, rc[i], delta, rho_l, rho_v, &fn, &du[i]);
        for (int k = 0; k < 3; ++k) f[k * n + i] = fn * g[k];
    }
    free(phi);
}

/* ---- velocity-Verlet steps (Eq. 1-2) ----------------------------------------------------
 * On entry f holds the forces of the current state and rc its cutoffs; k0 is the index of
 * the force evaluation that produced f. Each step: v += (dt/2m) f; x += dt v; wrap; the
 * force evaluation k = k0 + s first re-detects the interface when k % detect_every == 0;
 * forces; v += (dt/2m) f; record KE = m/2 sum v^2, PE = sum e_i, W = sum W_i. With the
 * thermostat on, half a thermostat step comes before the first kick and after the second;
 * nh = {xi, eta} carries its state in and out (left alone otherwise). */
int orc_run(const orc_params *p, int64_t n, double *x, double *v, double *rc, double *f,
            int64_t k0, int32_t nsteps, int32_t method, double nh[2], orc_thermo *th)
{
    int32_t d[3]; double h[3];
    orc_grid(p, d, h);
    int64_t G = (int64_t)d[0] * d[1] * d[2];
    double hdt = 0.5 * p->dt / p->mass;
    double *e = (double *)malloc(sizeof(double) * (size_t)n);
    double *w = (double *)malloc(sizeof(double) * (size_t)n * 6);
    int64_t *np = (int64_t *)malloc(sizeof(int64_t) * (size_t)n);
    orc_detect_out o;
    o.count = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)G);
    o.smooth = (uint32_t *)malloc(sizeof(uint32_t) * (size_t)G);
    o.raw = (uint8_t *)malloc((size_t)G);
    o.label = (uint8_t *)malloc((size_t)G);
    o.dist = (double *)malloc(sizeof(double) * (size_t)G);
    o.d = (double *)malloc(sizeof(double) * (size_t)n);
    o.dist_v = (p->tail || p->vapor_cutoff) ? (double *)malloc(sizeof(double) * (size_t)G) : NULL;
    double *ft = p->tail ? (double *)malloc(sizeof(double) * (size_t)n * 3) : NULL;
    double *du = p->tail ? (double *)malloc(sizeof(double) * (size_t)n) : NULL;
    if (p->tail) {
        /* the tail correction needs the fields of a detection: those of the entry state (the
         * cutoffs passed in rc are kept) */
        o.rc = o.d;
        orc_detect(p, n, x, &o);
    }
    o.rc = rc;
    for (int32_t s = 1; s <= nsteps; ++s) {
        int64_t k = k0 + s;
        if (p->thermostat) nh_half_step(p, n, v, nh);
        for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + hdt * f[i];
        for (int64_t i = 0; i < 3 * n; ++i) x[i] = x[i] + p->dt * v[i];
        orc_wrap(p, n, x);
        if (p->detect_every > 0 && k % p->detect_every == 0) orc_detect(p, n, x, &o);
        orc_forces(p, n, x, rc, n, NULL, method, f, e, w, np);
        if (p->tail) {
            orc_tail(p, o.dist, o.dist_v, o.km, n, x, rc, ft, du);
            for (int64_t i = 0; i < 3 * n; ++i) f[i] += ft[i];
            for (int64_t i = 0; i < n; ++i) e[i] += 0.5 * du[i];
        }
        for (int64_t i = 0; i < 3 * n; ++i) v[i] = v[i] + hdt * f[i];
        if (p->thermostat) nh_half_step(p, n, v, nh);
        if (th) {
            orc_thermo *t = &th[s - 1];
            memset(t, 0, sizeof *t);
            t->ke = kinetic(p, n, v);
            for (int64_t i = 0; i < n; ++i) {
                t->pe += e[i];
                for (int c = 0; c < 6; ++c) t->virial[c] += w[c * n + i];
                t->pairs += np[i];
            }
            t->step = k;
            t->xi = nh[0];
            t->eta = nh[1];
        }
    }
    free(e); free(w); free(np);
    free(o.count); free(o.smooth); free(o.raw); free(o.label); free(o.dist); free(o.d);
    free(o.dist_v); free(ft); free(du);
    return 0;
}
