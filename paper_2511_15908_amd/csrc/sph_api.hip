// C ABI of the SPH hot path (include/sph.h): validation, workspace carving,
// scene upload, the step sequence and host readback.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <string>
#include <vector>

#include "../../include/sph.h"
#include "sph_internal.h"

using namespace sphk;

namespace {

constexpr uint32_t kPhases = 10;
const char *kPhaseNames[kPhases] = {"place",   "keys",   "sort",   "reorder",  "springs",
                                    "density", "forces", "wrench", "integrate", "probes"};

struct Carve {
    char *base;
    size_t off = 0;
    template <typename P>
    P *take(size_t bytes)
    {
        off = (off + 255) & ~size_t(255);
        P *p = base ? reinterpret_cast<P *>(base + off) : nullptr;
        off += bytes ? bytes : 1;
        return p;
    }
};


}  // namespace

struct sph_ctx {
    sph_params prm{};
    int prec = 0;
    uint32_t n = 0, n_fluid = 0, n_soft = 0, n_bnd = 0;
    uint32_t nb = 0, nk = 0, n_objects = 0, rows = 0, nsprings = 0, nblk_w = 0, K = 1;
    std::vector<int32_t> kin_of_object;   // object -> kinematic index or -1
    std::vector<uint32_t> kin_objects;    // kinematic index -> object
    Grid grid{};
    double cell_size = 0;
    Phys<float> phf{};
    Phys<double> phd{};
    hipStream_t stream = nullptr;
    // device buffers
    void *pos[2] = {nullptr, nullptr}, *vel[2] = {nullptr, nullptr};
    uint32_t *id[2] = {nullptr, nullptr}, *aux[2] = {nullptr, nullptr};
    int cur = 0;
    Sort sort{};
    uint32_t *sorted_keys = nullptr, *sorted_vals = nullptr;
    uint32_t *inv_perm = nullptr, *cstart = nullptr, *cend = nullptr;
    void *dens = nullptr, *force = nullptr, *fspring = nullptr;
    uint64_t *masks = nullptr;
    uint32_t *row_id = nullptr, *row_ptr = nullptr, *partner = nullptr;
    double *sprm = nullptr;
    uint32_t *slot_id = nullptr, *slot_obj = nullptr;
    double *r_loc = nullptr, *poses = nullptr, *fbody = nullptr, *partials = nullptr;
    uint32_t *blk_obj = nullptr, *blk_first = nullptr, *blk_count = nullptr, *obj_blk0 = nullptr;
    double *ring = nullptr;
    uint32_t *ring_count = nullptr;
    uint32_t *err = nullptr;
    unsigned long long *stats = nullptr;
    int32_t *obj_of_id = nullptr;
    uint32_t max_probes = 0, n_probes = 0;
    double *probe_pts = nullptr, *probe_out = nullptr;
    int32_t *probe_frame = nullptr;
    std::vector<double> probe_host_pts;
    std::vector<int32_t> probe_host_frame;
    uint64_t steps = 0;
    bool dead = false;
    std::string last_error;
    std::vector<uint8_t> type_of_id;      // host copy of types (read_field)
    // profiling
    uint32_t prof_left = 0;
    std::vector<hipEvent_t> prof_ev;      // pairs per (step, phase)
    std::vector<int> prof_phase;
    size_t prof_used = 0;
    double prof_ms[kPhases] = {0};
    uint32_t prof_cnt[kPhases] = {0};
};

namespace {

sph_status dev_fail(sph_ctx *c, hipError_t e, const char *what)
{
    if (c) {
        c->dead = true;
        c->last_error = std::string(what) + ": " + hipGetErrorString(e);
    }
    return SPH_ERR_DEVICE;
}

#define HIPCHK(ctx, call)                                   \
    do {                                                    \
        hipError_t e_ = (call);                             \
        if (e_ != hipSuccess) return dev_fail(ctx, e_, #call); \
    } while (0)

bool finite3(const double *v) { return isfinite(v[0]) && isfinite(v[1]) && isfinite(v[2]); }

struct Plan {
    uint32_t n, nb, nk, rows, nsp2, nblk_w, nslots, K, nblk_sort, max_probes;
    int prec;
};

// Validate params and scene and derive the sizes the workspace depends on.
sph_status validate(const sph_params *p, const sph_scene *s, Plan &pl, std::string &why, Grid *gout,
                    double *cs_out)
{
    if (!p || !s) {
        why = "null params or scene";
        return SPH_ERR_ARG;
    }
    if (p->abi_version != SPH_ABI_VERSION) {
        why = "abi_version mismatch";
        return SPH_ERR_ARG;
    }
    for (uint32_t r : p->reserved)
        if (r) {
            why = "reserved fields must be zero";
            return SPH_ERR_ARG;
        }
    if (p->max_probes > (1u << 20)) {
        why = "max_probes must be <= 2^20";
        return SPH_ERR_ARG;
    }
    if (p->precision != SPH_FP32 && p->precision != SPH_FP64) {
        why = "precision must be SPH_FP32 or SPH_FP64";
        return SPH_ERR_ARG;
    }
    if (p->flags & ~7u) {
        why = "unknown flag bits";
        return SPH_ERR_UNSUPPORTED;
    }
    if (!(p->h > 0) || !isfinite(p->h) || !(p->rho0 > 0) || !isfinite(p->rho0) || !(p->k_pressure >= 0) ||
        !isfinite(p->k_pressure) || !(p->nu >= 0) || !isfinite(p->nu) || !(p->dt > 0) || !isfinite(p->dt) ||
        !finite3(p->gravity) || !(p->v_max >= 0) || !isfinite(p->v_max)) {
        why = "h, rho0, dt must be > 0; k, nu, v_max >= 0; all finite";
        return SPH_ERR_ARG;
    }
    if (p->smoothing_window < 1) {
        why = "smoothing_window must be >= 1";
        return SPH_ERR_ARG;
    }
    for (int a = 0; a < 3; ++a)
        if (!isfinite(p->domain_lo[a]) || !isfinite(p->domain_hi[a]) || !(p->domain_hi[a] > p->domain_lo[a])) {
            why = "domain_hi must exceed domain_lo on every axis";
            return SPH_ERR_ARG;
        }
    // grid
    const double R = 2.0 * p->h;
    const double cs = R * (1.0 + 1.0 / 1024.0);
    Grid g{};
    int maxd = 1;
    for (int a = 0; a < 3; ++a) {
        const double span = p->domain_hi[a] - p->domain_lo[a];
        const double dd = ceil(span / cs);
        if (dd > 1024.0) {
            why = "domain spans more than 1024 cells on an axis";
            return SPH_ERR_UNSUPPORTED;
        }
        int d = (int)dd;
        if (d < 1) d = 1;
        g.dims[a] = d;
        maxd = std::max(maxd, d);
        g.lo32[a] = (float)p->domain_lo[a];
        g.lo64[a] = p->domain_lo[a];
    }
    int bits = 0;
    while ((1 << bits) < maxd) ++bits;
    if (bits > 8) {
        why = "grid needs more than 2^24 Morton slots";
        return SPH_ERR_UNSUPPORTED;
    }
    g.bits = bits;
    g.nslots = 1u << (3 * bits);
    g.inv_cs64 = 1.0 / cs;
    g.inv_cs32 = (float)g.inv_cs64;
    const float Rf = (float)R;
    g.R2_32 = Rf * Rf;
    g.R2_64 = R * R;
    if (gout) *gout = g;
    if (cs_out) *cs_out = cs;
    // scene
    const uint32_t n = s->n;
    if (n > (1u << 24) - 1u) {
        why = "more than 2^24-1 particles";
        return SPH_ERR_UNSUPPORTED;
    }
    if (n && (!s->x || !s->v || !s->mass || !s->type || !s->object)) {
        why = "null scene array";
        return SPH_ERR_ARG;
    }
    if (s->n_objects && (!s->object_kinematic || !s->object_pose0)) {
        why = "null object array";
        return SPH_ERR_ARG;
    }
    uint32_t nk = 0, nb = 0, nsoft = 0;
    for (uint32_t o = 0; o < s->n_objects; ++o) {
        if (s->object_kinematic[o] > 1) {
            why = "object_kinematic must be 0 or 1";
            return SPH_ERR_ARG;
        }
        const double *pz = s->object_pose0 + 7 * o;
        double qn = 0;
        for (int k = 0; k < 7; ++k)
            if (!isfinite(pz[k])) {
                why = "non-finite object pose";
                return SPH_ERR_ARG;
            }
        for (int k = 3; k < 7; ++k) qn += pz[k] * pz[k];
        if (!(qn > 0)) {
            why = "zero quaternion";
            return SPH_ERR_ARG;
        }
        nk += s->object_kinematic[o];
    }
    std::vector<uint32_t> per_obj(s->n_objects, 0);
    for (uint32_t i = 0; i < n; ++i) {
        const uint8_t t = s->type[i];
        if (t > SPH_BOUNDARY) {
            why = "unknown particle type";
            return SPH_ERR_ARG;
        }
        for (int a = 0; a < 3; ++a)
            if (!isfinite(s->x[3 * i + a]) || !isfinite(s->v[3 * i + a])) {
                why = "non-finite position or velocity";
                return SPH_ERR_ARG;
            }
        if (t == SPH_BOUNDARY) {
            const int32_t o = s->object[i];
            if (o < 0 || (uint32_t)o >= s->n_objects) {
                why = "boundary particle with an invalid object id";
                return SPH_ERR_ARG;
            }
            per_obj[o]++;
            if (s->object_kinematic[o]) ++nb;
        } else {
            if (!(s->mass[i] > 0) || !isfinite(s->mass[i])) {
                why = "fluid/soft mass must be positive and finite";
                return SPH_ERR_ARG;
            }
            if (t == SPH_SOFT) ++nsoft;
        }
    }
    if (s->n_springs) {
        if (!s->spring_ij || !s->spring_L0 || !s->spring_k || !s->spring_c) {
            why = "null spring array";
            return SPH_ERR_ARG;
        }
        for (uint32_t k = 0; k < s->n_springs; ++k) {
            const uint32_t a = s->spring_ij[2 * k], b = s->spring_ij[2 * k + 1];
            if (a >= n || b >= n || a == b || s->type[a] != SPH_SOFT || s->type[b] != SPH_SOFT) {
                why = "spring ends must be two distinct soft particles";
                return SPH_ERR_ARG;
            }
            if (!isfinite(s->spring_L0[k]) || !isfinite(s->spring_k[k]) || !isfinite(s->spring_c[k]) ||
                s->spring_L0[k] < 0) {
                why = "spring parameters must be finite, L0 >= 0";
                return SPH_ERR_ARG;
            }
        }
    }
    uint32_t nblk_w = 0;
    for (uint32_t o = 0; o < s->n_objects; ++o)
        if (s->object_kinematic[o]) nblk_w += (per_obj[o] + 255) / 256;
    pl.n = n;
    pl.nb = nb;
    pl.nk = nk;
    pl.rows = nsoft;
    pl.nsp2 = 2 * s->n_springs;
    pl.nblk_w = nblk_w;
    pl.nslots = g.nslots;
    pl.K = p->smoothing_window;
    pl.nblk_sort = (n + 2047) / 2048;
    pl.prec = p->precision;
    pl.max_probes = p->max_probes;
    return SPH_OK;
}

void carve(sph_ctx *c, const Plan &pl, char *base, size_t *total)
{
    Carve cv{base};
    const size_t tsz = pl.prec == SPH_FP64 ? 8 : 4;
    const size_t n = pl.n;
    for (int b = 0; b < 2; ++b) {
        c->pos[b] = cv.take<void>(n * 4 * tsz);
        c->vel[b] = cv.take<void>(n * 4 * tsz);
        c->id[b] = cv.take<uint32_t>(n * 4);
        c->aux[b] = cv.take<uint32_t>(n * 4);
    }
    c->sort.keys_a = cv.take<uint32_t>(n * 4);
    c->sort.keys_b = cv.take<uint32_t>(n * 4);
    c->sort.vals_a = cv.take<uint32_t>(n * 4);
    c->sort.vals_b = cv.take<uint32_t>(n * 4);
    c->sort.hist = cv.take<uint32_t>((size_t)256 * std::max<uint32_t>(pl.nblk_sort, 1) * 4);
    c->sort.dbase = cv.take<uint32_t>(256 * 4);
    c->sort.nblk = pl.nblk_sort;
    c->inv_perm = cv.take<uint32_t>(n * 4);
    c->cstart = cv.take<uint32_t>((size_t)pl.nslots * 4);
    c->cend = cv.take<uint32_t>((size_t)pl.nslots * 4);
    c->dens = cv.take<void>(n * 2 * tsz);
    c->force = cv.take<void>(n * 4 * tsz);
    c->masks = cv.take<uint64_t>((size_t)kMaxWords * n * 8);
    c->fspring = cv.take<void>((size_t)pl.rows * 4 * tsz);
    c->row_id = cv.take<uint32_t>((size_t)pl.rows * 4);
    c->row_ptr = cv.take<uint32_t>((size_t)(pl.rows + 1) * 4);
    c->partner = cv.take<uint32_t>((size_t)pl.nsp2 * 4);
    c->sprm = cv.take<double>((size_t)pl.nsp2 * 3 * 8);
    c->slot_id = cv.take<uint32_t>((size_t)pl.nb * 4);
    c->slot_obj = cv.take<uint32_t>((size_t)pl.nb * 4);
    c->r_loc = cv.take<double>((size_t)pl.nb * 3 * 8);
    c->fbody = cv.take<double>((size_t)pl.nb * 3 * 8);
    c->partials = cv.take<double>((size_t)pl.nblk_w * 6 * 8);
    c->blk_obj = cv.take<uint32_t>((size_t)pl.nblk_w * 4);
    c->blk_first = cv.take<uint32_t>((size_t)pl.nblk_w * 4);
    c->blk_count = cv.take<uint32_t>((size_t)pl.nblk_w * 4);
    c->obj_blk0 = cv.take<uint32_t>((size_t)(pl.nk + 1) * 4);
    c->poses = cv.take<double>((size_t)pl.nk * 16 * 8);
    c->ring = cv.take<double>((size_t)pl.nk * pl.K * 6 * 8);
    c->ring_count = cv.take<uint32_t>((size_t)pl.nk * 4);
    c->err = cv.take<uint32_t>(16);
    c->stats = cv.take<unsigned long long>(8 * 8);
    c->obj_of_id = cv.take<int32_t>(n * 4);
    c->probe_pts = cv.take<double>((size_t)pl.max_probes * 3 * 8);
    c->probe_frame = cv.take<int32_t>((size_t)pl.max_probes * 4);
    c->probe_out = cv.take<double>((size_t)pl.max_probes * 8);
    *total = cv.off + 256;
}

template <typename T>
State<T> state(sph_ctx *c, int b)
{
    return State<T>{(V4<T> *)c->pos[b], (V4<T> *)c->vel[b], c->id[b], c->aux[b]};
}

BodyArgs body_args(sph_ctx *c)
{
    BodyArgs b{};
    b.nb = c->nb;
    b.slot_id = c->slot_id;
    b.slot_obj = c->slot_obj;
    b.r_loc = c->r_loc;
    b.poses = c->poses;
    b.fbody = c->fbody;
    b.partials = c->partials;
    b.blk_obj = c->blk_obj;
    b.blk_first = c->blk_first;
    b.blk_count = c->blk_count;
    b.obj_blk0 = c->obj_blk0;
    b.nblk = c->nblk_w;
    b.nk = c->nk;
    b.ring = c->ring;
    b.ring_count = c->ring_count;
    b.K = c->K;
    b.dt = c->prm.dt;
    return b;
}

void prof_mark(sph_ctx *c, int phase, bool begin)
{
    if (!c->prof_left) return;
    if (c->prof_used >= c->prof_ev.size()) return;
    (void)hipEventRecord(c->prof_ev[c->prof_used], c->stream);
    if (begin) c->prof_phase[c->prof_used / 2] = phase;
    ++c->prof_used;
}

// Neighbour search: keys, radix sort, cell table, reorder into the other buffer.
template <typename T>
void neighbour_search(sph_ctx *c)
{
    const uint32_t n = c->n;
    prof_mark(c, 1, true);
    launch_keys<T>(c->stream, n, (const V4<T> *)c->pos[c->cur], c->grid, c->sort.keys_a);
    prof_mark(c, 1, false);
    prof_mark(c, 2, true);
    launch_radix_sort(c->stream, n, 3 * c->grid.bits, c->sort, &c->sorted_keys, &c->sorted_vals);
    prof_mark(c, 2, false);
    prof_mark(c, 3, true);
    launch_clear_u32(c->stream, c->cstart, c->grid.nslots);
    launch_clear_u32(c->stream, c->cend, c->grid.nslots);
    launch_reorder<T>(c->stream, n, c->sorted_vals, c->sorted_keys, state<T>(c, c->cur), state<T>(c, 1 - c->cur),
                      c->inv_perm, c->cstart, c->cend);
    c->cur = 1 - c->cur;
    prof_mark(c, 3, false);
}

template <typename T>
const Phys<T> &phys(const sph_ctx *c);
template <>
const Phys<float> &phys<float>(const sph_ctx *c) { return c->phf; }
template <>
const Phys<double> &phys<double>(const sph_ctx *c) { return c->phd; }

template <typename T>
void one_step(sph_ctx *c)
{
    hipStream_t s = c->stream;
    const BodyArgs ba = body_args(c);
    prof_mark(c, 0, true);
    launch_place<T>(s, ba, c->inv_perm, state<T>(c, c->cur));
    prof_mark(c, 0, false);
    neighbour_search<T>(c);
    const State<T> st = state<T>(c, c->cur);
    prof_mark(c, 4, true);
    SpringArgs sa{c->rows, c->row_id, c->row_ptr, c->partner, c->sprm};
    launch_springs<T>(s, sa, c->inv_perm, st, (V4<T> *)c->fspring);
    prof_mark(c, 4, false);
    prof_mark(c, 5, true);
    launch_density<T>(s, c->n, st, c->grid, phys<T>(c), c->cstart, c->cend, (V2<T> *)c->dens, c->masks, c->err,
                     c->stats);
    prof_mark(c, 5, false);
    prof_mark(c, 6, true);
    launch_forces<T>(s, c->n, st, c->grid, phys<T>(c), c->cstart, c->cend, (const V2<T> *)c->dens, c->masks,
                     (const V4<T> *)c->fspring, (V4<T> *)c->force, c->fbody, c->err, c->stats);
    prof_mark(c, 6, false);
    prof_mark(c, 9, true);
    if (c->n_probes) {
        ProbeArgs pa{c->n_probes, c->probe_pts, c->probe_frame, c->poses, c->probe_out};
        launch_probe<T>(s, pa, st, c->grid, phys<T>(c), c->cstart, c->cend);
    }
    prof_mark(c, 9, false);
    prof_mark(c, 7, true);
    launch_wrench(s, ba);
    prof_mark(c, 7, false);
    prof_mark(c, 8, true);
    launch_integrate<T>(s, c->n, st, (const V4<T> *)c->force, phys<T>(c), c->err);
    prof_mark(c, 8, false);
    if (c->prof_left) --c->prof_left;
    ++c->steps;
}

template <typename T>
void fill_phys(Phys<T> &ph, const sph_params *p)
{
    const double h = p->h;
    const double alpha = 3.0 / (2.0 * M_PI * h * h * h);
    ph.inv_h = (T)(1.0 / h);
    ph.alpha6 = (T)(alpha / 6.0);
    ph.gc = (T)(alpha / (2.0 * h * h));
    ph.gch = (T)(alpha / (2.0 * h));
    ph.eps = (T)(0.01 * h * h);
    ph.two_nu = (T)(2.0 * p->nu);
    ph.gx = (T)p->gravity[0];
    ph.gy = (T)p->gravity[1];
    ph.gz = (T)p->gravity[2];
    ph.dt = (T)p->dt;
    ph.vmax2 = (T)(p->v_max * p->v_max);
    ph.rho0 = p->rho0;
    ph.kp = p->k_pressure;
    ph.psi_scale = p->rho0;
    ph.inv_h64 = 1.0 / h;
    ph.alpha6_64 = alpha / 6.0;
    ph.flags = p->flags;
}

void quat_normalise(const double *q, double *out)
{
    const double s = sqrt(q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3]);
    for (int k = 0; k < 4; ++k) out[k] = q[k] / s;
}

void quat_to_R(const double *q, double R[9])
{
    const double w = q[0], x = q[1], y = q[2], z = q[3];
    R[0] = 1.0 - 2.0 * (y * y + z * z);
    R[1] = 2.0 * (x * y - w * z);
    R[2] = 2.0 * (x * z + w * y);
    R[3] = 2.0 * (x * y + w * z);
    R[4] = 1.0 - 2.0 * (x * x + z * z);
    R[5] = 2.0 * (y * z - w * x);
    R[6] = 2.0 * (x * z - w * y);
    R[7] = 2.0 * (y * z + w * x);
    R[8] = 1.0 - 2.0 * (x * x + y * y);
}

template <typename T>
sph_status upload(sph_ctx *c, const sph_scene *s)
{
    const uint32_t n = c->n;
    hipStream_t st = c->stream;
    std::vector<V4<T>> pos(n), vel(n);
    std::vector<uint32_t> ids(n), aux(n);
    std::vector<int32_t> obj(n);
    // soft rows and springs
    std::vector<uint32_t> row_of(n, 0xffffffffu), row_id;
    for (uint32_t i = 0; i < n; ++i)
        if (s->type[i] == SPH_SOFT) {
            row_of[i] = (uint32_t)row_id.size();
            row_id.push_back(i);
        }
    std::vector<uint32_t> rcount(c->rows + 1, 0);
    for (uint32_t k = 0; k < s->n_springs; ++k) {
        rcount[row_of[s->spring_ij[2 * k]] + 1]++;
        rcount[row_of[s->spring_ij[2 * k + 1]] + 1]++;
    }
    for (uint32_t r = 0; r < c->rows; ++r) rcount[r + 1] += rcount[r];
    std::vector<uint32_t> row_ptr(rcount), fillp(rcount.begin(), rcount.end() - 1);
    std::vector<uint32_t> partner(2 * s->n_springs);
    std::vector<double> sprm(6 * (size_t)s->n_springs);
    for (uint32_t k = 0; k < s->n_springs; ++k) {
        const uint32_t a = s->spring_ij[2 * k], b = s->spring_ij[2 * k + 1];
        const uint32_t ea = fillp[row_of[a]]++, eb = fillp[row_of[b]]++;
        partner[ea] = b;
        partner[eb] = a;
        for (uint32_t e : {ea, eb}) {
            sprm[3 * e] = s->spring_L0[k];
            sprm[3 * e + 1] = s->spring_k[k];
            sprm[3 * e + 2] = s->spring_c[k];
        }
    }
    // kinematic bodies: slots ordered by kinematic index then particle id
    std::vector<uint32_t> slot_id, slot_obj, blk_obj, blk_first, blk_count, obj_blk0;
    std::vector<double> r_loc, poses(16 * (size_t)c->nk, 0.0);
    std::vector<uint32_t> slot_of(n, 0);
    for (uint32_t k = 0; k < c->nk; ++k) {
        const uint32_t o = c->kin_objects[k];
        const double *pz = s->object_pose0 + 7 * o;
        double q[4], R[9];
        quat_normalise(pz + 3, q);
        quat_to_R(q, R);
        for (int a = 0; a < 3; ++a) poses[16 * k + a] = pz[a];
        for (int a = 0; a < 4; ++a) poses[16 * k + 3 + a] = q[a];
        obj_blk0.push_back((uint32_t)blk_obj.size());
        const uint32_t first = (uint32_t)slot_id.size();
        for (uint32_t i = 0; i < n; ++i) {
            if (s->type[i] != SPH_BOUNDARY || s->object[i] != (int32_t)o) continue;
            slot_of[i] = (uint32_t)slot_id.size();
            slot_id.push_back(i);
            slot_obj.push_back(k);
            const double d[3] = {s->x[3 * i] - pz[0], s->x[3 * i + 1] - pz[1], s->x[3 * i + 2] - pz[2]};
            for (int a = 0; a < 3; ++a) r_loc.push_back(R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2]);
        }
        const uint32_t cnt = (uint32_t)slot_id.size() - first;
        for (uint32_t b0 = 0; b0 < cnt; b0 += 256) {
            blk_obj.push_back(k);
            blk_first.push_back(first + b0);
            blk_count.push_back(std::min<uint32_t>(256, cnt - b0));
        }
    }
    obj_blk0.push_back((uint32_t)blk_obj.size());
    for (uint32_t i = 0; i < n; ++i) {
        const uint8_t t = s->type[i];
        pos[i] = V4<T>{(T)s->x[3 * i], (T)s->x[3 * i + 1], (T)s->x[3 * i + 2],
                       t == SPH_BOUNDARY ? (T)0 : (T)s->mass[i]};
        vel[i] = V4<T>{(T)s->v[3 * i], (T)s->v[3 * i + 1], (T)s->v[3 * i + 2], (T)0};
        ids[i] = i;
        obj[i] = t == SPH_BOUNDARY ? s->object[i] : -1;
        if (t == SPH_FLUID)
            aux[i] = aux_make(TY_FLUID, false, 0);
        else if (t == SPH_SOFT)
            aux[i] = aux_make(TY_SOFT, false, row_of[i]);
        else if (c->kin_of_object[s->object[i]] >= 0)
            aux[i] = aux_make(TY_BOUNDARY, true, slot_of[i]);
        else
            aux[i] = aux_make(TY_BOUNDARY, false, (uint32_t)s->object[i]);
    }
    auto H2D = [&](void *dst, const void *src, size_t bytes) -> hipError_t {
        if (!bytes) return hipSuccess;
        return hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st);
    };
    const int b = 0;
    HIPCHK(c, H2D(c->pos[b], pos.data(), pos.size() * sizeof(V4<T>)));
    HIPCHK(c, H2D(c->vel[b], vel.data(), vel.size() * sizeof(V4<T>)));
    HIPCHK(c, H2D(c->id[b], ids.data(), ids.size() * 4));
    HIPCHK(c, H2D(c->aux[b], aux.data(), aux.size() * 4));
    HIPCHK(c, H2D(c->obj_of_id, obj.data(), obj.size() * 4));
    HIPCHK(c, H2D(c->row_id, row_id.data(), row_id.size() * 4));
    HIPCHK(c, H2D(c->row_ptr, row_ptr.data(), row_ptr.size() * 4));
    HIPCHK(c, H2D(c->partner, partner.data(), partner.size() * 4));
    HIPCHK(c, H2D(c->sprm, sprm.data(), sprm.size() * 8));
    HIPCHK(c, H2D(c->slot_id, slot_id.data(), slot_id.size() * 4));
    HIPCHK(c, H2D(c->slot_obj, slot_obj.data(), slot_obj.size() * 4));
    HIPCHK(c, H2D(c->r_loc, r_loc.data(), r_loc.size() * 8));
    HIPCHK(c, H2D(c->blk_obj, blk_obj.data(), blk_obj.size() * 4));
    HIPCHK(c, H2D(c->blk_first, blk_first.data(), blk_first.size() * 4));
    HIPCHK(c, H2D(c->blk_count, blk_count.data(), blk_count.size() * 4));
    HIPCHK(c, H2D(c->obj_blk0, obj_blk0.data(), obj_blk0.size() * 4));
    HIPCHK(c, H2D(c->poses, poses.data(), poses.size() * 8));
    // zero what must start at zero (fill kernels, no memset nodes)
    launch_clear_u32(st, c->ring_count, c->nk);
    launch_clear_u32(st, c->err, 4);
    launch_clear_u32(st, (uint32_t *)c->stats, 16);
    launch_clear_u32(st, (uint32_t *)c->dens, (size_t)n * 2 * sizeof(T) / 4);
    launch_clear_u32(st, (uint32_t *)c->force, (size_t)n * 4 * sizeof(T) / 4);
    launch_clear_u32(st, (uint32_t *)c->fspring, (size_t)c->rows * 4 * sizeof(T) / 4);
    launch_clear_u32(st, (uint32_t *)c->fbody, (size_t)c->nb * 6);
    // first neighbour search, then boundary volumes from the initial configuration
    c->cur = 0;
    if (n) {
        neighbour_search<T>(c);
        launch_psi_obj<T>(st, n, state<T>(c, c->cur), c->grid, phys<T>(c), c->cstart, c->cend, c->obj_of_id);
    }
    HIPCHK(c, hipGetLastError());
    HIPCHK(c, hipStreamSynchronize(st));
    c->type_of_id.assign(s->type, s->type + n);
    return SPH_OK;
}

sph_status check_err(sph_ctx *c)
{
    uint32_t e = 0;
    HIPCHK(c, hipMemcpyAsync(&e, c->err, 4, hipMemcpyDeviceToHost, c->stream));
    HIPCHK(c, hipStreamSynchronize(c->stream));
    if (e) {
        const uint32_t z = 0;
        HIPCHK(c, hipMemcpyAsync(c->err, &z, 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (e & ERR_CAPACITY) {
            c->last_error = "a cell neighbourhood exceeded the candidate capacity";
            return SPH_ERR_CAPACITY;
        }
        c->last_error = "non-finite or over-speed particle";
        return SPH_ERR_UNSTABLE;
    }
    return SPH_OK;
}

}  // namespace

extern "C" {

const char *sph_status_string(sph_status s)
{
    switch (s) {
    case SPH_OK: return "ok";
    case SPH_ERR_ARG: return "invalid argument";
    case SPH_ERR_WORKSPACE: return "workspace missing, misaligned or too small";
    case SPH_ERR_DEVICE: return "HIP runtime error";
    case SPH_ERR_STATE: return "context unusable after an earlier device error";
    case SPH_ERR_UNSTABLE: return "simulation became unstable";
    case SPH_ERR_UNSUPPORTED: return "unsupported configuration";
    case SPH_ERR_CAPACITY: return "neighbourhood capacity exceeded";
    }
    return "unknown status";
}

const char *sph_last_error(const sph_ctx *ctx)
{
    if (!ctx) return "null context";
    return ctx->last_error.c_str();
}

const char *sph_profile_phase_name(uint32_t phase) { return phase < kPhases ? kPhaseNames[phase] : nullptr; }

sph_status sph_workspace_size(const sph_params *params, const sph_scene *scene, size_t *bytes)
{
    if (!bytes) return SPH_ERR_ARG;
    Plan pl{};
    std::string why;
    sph_status st = validate(params, scene, pl, why, nullptr, nullptr);
    if (st != SPH_OK) return st;
    sph_ctx tmp;
    carve(&tmp, pl, nullptr, bytes);
    return SPH_OK;
}

sph_status sph_init(const sph_params *params, const sph_scene *scene, void *d_workspace, size_t ws_bytes,
                    void *hip_stream, sph_ctx **out)
{
    if (!out) return SPH_ERR_ARG;
    *out = nullptr;
    Plan pl{};
    std::string why;
    Grid g{};
    double cs = 0;
    sph_status st = validate(params, scene, pl, why, &g, &cs);
    if (st != SPH_OK) return st;
    size_t need = 0;
    {
        sph_ctx tmp;
        carve(&tmp, pl, nullptr, &need);
    }
    if (!d_workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255u)) return SPH_ERR_WORKSPACE;
    sph_ctx *c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_ERR_DEVICE;
    c->prm = *params;
    c->prec = params->precision;
    c->n = pl.n;
    c->nb = pl.nb;
    c->nk = pl.nk;
    c->rows = pl.rows;
    c->nsprings = scene->n_springs;
    c->nblk_w = pl.nblk_w;
    c->K = pl.K;
    c->n_objects = scene->n_objects;
    c->max_probes = pl.max_probes;
    c->grid = g;
    c->cell_size = cs;
    c->stream = (hipStream_t)hip_stream;
    c->kin_of_object.assign(scene->n_objects, -1);
    for (uint32_t o = 0; o < scene->n_objects; ++o)
        if (scene->object_kinematic[o]) {
            c->kin_of_object[o] = (int32_t)c->kin_objects.size();
            c->kin_objects.push_back(o);
        }
    for (uint32_t i = 0; i < scene->n; ++i) {
        if (scene->type[i] == SPH_FLUID) ++c->n_fluid;
        else if (scene->type[i] == SPH_SOFT) ++c->n_soft;
        else ++c->n_bnd;
    }
    fill_phys(c->phf, params);
    fill_phys(c->phd, params);
    size_t total = 0;
    carve(c, pl, (char *)d_workspace, &total);
    sph_status r = c->prec == SPH_FP64 ? upload<double>(c, scene) : upload<float>(c, scene);
    if (r != SPH_OK) {
        delete c;
        return r;
    }
    *out = c;
    return SPH_OK;
}

sph_status sph_set_body_pose(sph_ctx *ctx, uint32_t object, const double c[3], const double q[4], const double v[3],
                             const double w[3])
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (!c || !q || !v || !w || object >= ctx->n_objects || ctx->kin_of_object[object] < 0) return SPH_ERR_ARG;
    if (!finite3(c) || !finite3(v) || !finite3(w) || !isfinite(q[0]) || !isfinite(q[1]) || !isfinite(q[2]) ||
        !isfinite(q[3]))
        return SPH_ERR_ARG;
    const double qn = q[0] * q[0] + q[1] * q[1] + q[2] * q[2] + q[3] * q[3];
    if (!(qn > 0)) return SPH_ERR_ARG;
    double qq[4];
    quat_normalise(q, qq);
    launch_set_pose(ctx->stream, ctx->poses + 16 * ctx->kin_of_object[object], c, qq, v, w);
    HIPCHK(ctx, hipGetLastError());
    return SPH_OK;
}

sph_status sph_step(sph_ctx *ctx, uint32_t n_steps, void *hip_stream)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    ctx->stream = (hipStream_t)hip_stream;
    if (!ctx->n) {
        ctx->steps += n_steps;
        return SPH_OK;
    }
    for (uint32_t k = 0; k < n_steps; ++k) {
        if (ctx->prec == SPH_FP64)
            one_step<double>(ctx);
        else
            one_step<float>(ctx);
    }
    HIPCHK(ctx, hipGetLastError());
    return SPH_OK;
}

sph_status sph_synchronize(sph_ctx *ctx)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    return check_err(ctx);
}

sph_status sph_get_body_wrench(sph_ctx *ctx, uint32_t object, double F[3], double T[3], int smoothed)
{
    if (!ctx || !F || !T) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (object >= ctx->n_objects || ctx->kin_of_object[object] < 0) return SPH_ERR_ARG;
    const uint32_t k = (uint32_t)ctx->kin_of_object[object];
    std::vector<double> ring((size_t)ctx->K * 6);
    uint32_t cnt = 0;
    HIPCHK(ctx, hipMemcpyAsync(ring.data(), ctx->ring + (size_t)k * ctx->K * 6, ring.size() * 8,
                               hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipMemcpyAsync(&cnt, ctx->ring_count + k, 4, hipMemcpyDeviceToHost, ctx->stream));
    sph_status st = check_err(ctx);
    if (st == SPH_ERR_DEVICE) return st;
    double out[6] = {0, 0, 0, 0, 0, 0};
    if (cnt) {
        if (!smoothed) {
            const double *s = ring.data() + (size_t)((cnt - 1) % ctx->K) * 6;
            for (int a = 0; a < 6; ++a) out[a] = s[a];
        } else {
            const uint32_t m = std::min(cnt, ctx->K);
            for (uint32_t j = 0; j < m; ++j) {       // oldest to newest
                const uint32_t idx = (cnt - m + j) % ctx->K;
                for (int a = 0; a < 6; ++a) out[a] += ring[(size_t)idx * 6 + a];
            }
            for (int a = 0; a < 6; ++a) out[a] /= (double)m;
        }
    }
    for (int a = 0; a < 3; ++a) {
        F[a] = out[a];
        T[a] = out[3 + a];
    }
    return st;
}

sph_status sph_set_probes(sph_ctx *ctx, uint32_t n, const double *points, const int32_t *frame)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (n > ctx->max_probes || (n && (!points || !frame))) return SPH_ERR_ARG;
    std::vector<double> pts(points, points + 3 * (size_t)n);
    std::vector<int32_t> fr(n);
    for (uint32_t i = 0; i < n; ++i) {
        if (!finite3(points + 3 * i)) return SPH_ERR_ARG;
        if (frame[i] < 0) {
            fr[i] = -1;
        } else {
            if ((uint32_t)frame[i] >= ctx->n_objects || ctx->kin_of_object[frame[i]] < 0) return SPH_ERR_ARG;
            fr[i] = ctx->kin_of_object[frame[i]];
        }
    }
    // the previous upload may still read the host copies
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    ctx->probe_host_pts.swap(pts);
    ctx->probe_host_frame.swap(fr);
    if (n) {
        HIPCHK(ctx, hipMemcpyAsync(ctx->probe_pts, ctx->probe_host_pts.data(), 24 * (size_t)n,
                                   hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(ctx->probe_frame, ctx->probe_host_frame.data(), 4 * (size_t)n,
                                   hipMemcpyHostToDevice, ctx->stream));
        launch_clear_u32(ctx->stream, (uint32_t *)ctx->probe_out, 2 * (size_t)n);
    }
    ctx->n_probes = n;
    HIPCHK(ctx, hipGetLastError());
    return SPH_OK;
}

sph_status sph_read_probes(sph_ctx *ctx, double *rho, uint32_t n)
{
    if (!ctx || (n && !rho)) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (n != ctx->n_probes) return SPH_ERR_ARG;
    if (n) HIPCHK(ctx, hipMemcpyAsync(rho, ctx->probe_out, 8 * (size_t)n, hipMemcpyDeviceToHost, ctx->stream));
    return check_err(ctx);
}

sph_status sph_reset_smoothing(sph_ctx *ctx, uint32_t object)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (object >= ctx->n_objects || ctx->kin_of_object[object] < 0) return SPH_ERR_ARG;
    launch_reset_ring(ctx->stream, ctx->ring_count + ctx->kin_of_object[object]);
    HIPCHK(ctx, hipGetLastError());
    return SPH_OK;
}

}  // extern "C"

namespace {

template <typename T>
sph_status read_field_t(sph_ctx *c, int field, void *dst, size_t bytes)
{
    const uint32_t n = c->n;
    const size_t want = (field == SPH_FIELD_KEY) ? (size_t)n * 4
                        : (field == SPH_FIELD_X || field == SPH_FIELD_V || field == SPH_FIELD_FORCE ||
                           field == SPH_FIELD_SPRING)
                            ? (size_t)n * 3 * 8
                            : (size_t)n * 8;
    if (field < SPH_FIELD_X || field > SPH_FIELD_SPRING) return SPH_ERR_ARG;
    if (bytes != want || (!dst && bytes)) return SPH_ERR_ARG;
    if (!n) return check_err(c);
    hipStream_t s = c->stream;
    std::vector<uint32_t> ids(n), aux(n);
    HIPCHK(c, hipMemcpyAsync(ids.data(), c->id[c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
    HIPCHK(c, hipMemcpyAsync(aux.data(), c->aux[c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
    std::vector<V4<T>> v4;
    std::vector<V2<T>> v2;
    std::vector<uint32_t> keys;
    std::vector<double> fb;
    if (field == SPH_FIELD_X || field == SPH_FIELD_PSI) {
        v4.resize(n);
        HIPCHK(c, hipMemcpyAsync(v4.data(), c->pos[c->cur], (size_t)n * sizeof(V4<T>), hipMemcpyDeviceToHost, s));
    } else if (field == SPH_FIELD_V) {
        v4.resize(n);
        HIPCHK(c, hipMemcpyAsync(v4.data(), c->vel[c->cur], (size_t)n * sizeof(V4<T>), hipMemcpyDeviceToHost, s));
    } else if (field == SPH_FIELD_FORCE) {
        v4.resize(n);
        HIPCHK(c, hipMemcpyAsync(v4.data(), c->force, (size_t)n * sizeof(V4<T>), hipMemcpyDeviceToHost, s));
        fb.resize((size_t)c->nb * 3);
        if (c->nb)
            HIPCHK(c, hipMemcpyAsync(fb.data(), c->fbody, fb.size() * 8, hipMemcpyDeviceToHost, s));
    } else if (field == SPH_FIELD_SPRING) {
        v4.resize(c->rows);
        if (c->rows)
            HIPCHK(c, hipMemcpyAsync(v4.data(), c->fspring, (size_t)c->rows * sizeof(V4<T>), hipMemcpyDeviceToHost,
                                     s));
    } else if (field == SPH_FIELD_RHO || field == SPH_FIELD_PRESSURE) {
        v2.resize(n);
        HIPCHK(c, hipMemcpyAsync(v2.data(), c->dens, (size_t)n * sizeof(V2<T>), hipMemcpyDeviceToHost, s));
    } else if (field == SPH_FIELD_KEY) {
        keys.resize(n);
        HIPCHK(c, hipMemcpyAsync(keys.data(), c->sorted_keys, (size_t)n * 4, hipMemcpyDeviceToHost, s));
    }
    sph_status st = check_err(c);
    if (st == SPH_ERR_DEVICE) return st;
    double *d = (double *)dst;
    for (uint32_t p = 0; p < n; ++p) {
        const uint32_t i = ids[p];
        const uint32_t a = aux[p];
        const bool bnd = aux_type(a) == TY_BOUNDARY;
        switch (field) {
        case SPH_FIELD_X:
        case SPH_FIELD_V:
            d[3 * i] = (double)v4[p].x;
            d[3 * i + 1] = (double)v4[p].y;
            d[3 * i + 2] = (double)v4[p].z;
            break;
        case SPH_FIELD_FORCE:
            if (bnd && aux_kin(a)) {
                const size_t sl = aux_index(a);
                d[3 * i] = fb[3 * sl];
                d[3 * i + 1] = fb[3 * sl + 1];
                d[3 * i + 2] = fb[3 * sl + 2];
            } else if (bnd) {
                d[3 * i] = d[3 * i + 1] = d[3 * i + 2] = 0.0;
            } else {
                d[3 * i] = (double)v4[p].x;
                d[3 * i + 1] = (double)v4[p].y;
                d[3 * i + 2] = (double)v4[p].z;
            }
            break;
        case SPH_FIELD_SPRING:
            if (aux_type(a) == TY_SOFT) {
                const V4<T> &f = v4[aux_index(a)];
                d[3 * i] = (double)f.x;
                d[3 * i + 1] = (double)f.y;
                d[3 * i + 2] = (double)f.z;
            } else {
                d[3 * i] = d[3 * i + 1] = d[3 * i + 2] = 0.0;
            }
            break;
        case SPH_FIELD_RHO:
            d[i] = bnd ? 0.0 : (double)v2[p].x;
            break;
        case SPH_FIELD_PRESSURE: {
            double pr = bnd ? 0.0 : c->prm.k_pressure * ((double)v2[p].x - c->prm.rho0);
            if ((c->prm.flags & SPH_FLAG_CLAMP_NEG_PRESSURE) && pr < 0) pr = 0;
            d[i] = pr;
            break;
        }
        case SPH_FIELD_PSI:
            d[i] = bnd ? -(double)v4[p].w : 0.0;
            break;
        case SPH_FIELD_KEY:
            ((uint32_t *)dst)[i] = keys[p];
            break;
        }
    }
    return st;
}

template <typename T>
sph_status debug_nbrs_t(sph_ctx *c, uint32_t nt, const uint32_t *targets, uint32_t *counts, uint32_t *ids_out,
                        size_t cap, size_t *total)
{
    const uint32_t n = c->n;
    hipStream_t s = c->stream;
    std::vector<uint32_t> ids(n), aux(n), keys(n), cs(c->grid.nslots), ce(c->grid.nslots);
    std::vector<uint64_t> masks((size_t)kMaxWords * n);
    if (n) {
        HIPCHK(c, hipMemcpyAsync(ids.data(), c->id[c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(aux.data(), c->aux[c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(keys.data(), c->sorted_keys, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(cs.data(), c->cstart, cs.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ce.data(), c->cend, ce.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(masks.data(), c->masks, masks.size() * 8, hipMemcpyDeviceToHost, s));
    }
    sph_status st = check_err(c);
    if (st == SPH_ERR_DEVICE) return st;
    std::vector<std::vector<uint32_t>> lists(n);
    std::vector<uint8_t> want(n, targets ? 0 : 1);
    if (targets)
        for (uint32_t t = 0; t < nt; ++t) want[targets[t]] = 1;
    const Grid &g = c->grid;
    for (uint32_t p = 0; p < n; ++p) {
        if (!want[ids[p]]) continue;
        const uint32_t a = aux[p];
        if (aux_type(a) == TY_BOUNDARY && !aux_kin(a)) continue;
        const uint32_t home = keys[p];
        const int cx = (int)compact3(home), cy = (int)compact3(home >> 1), cz = (int)compact3(home >> 2);
        uint32_t start[27], cnt[27], L = 0;
        for (int k = 0; k < 27; ++k) {
            int ox, oy, oz;
            stencil_offset(k, ox, oy, oz);
            const int nx = cx + ox, ny = cy + oy, nz = cz + oz;
            uint32_t stt = 0, ct = 0;
            if (nx >= 0 && ny >= 0 && nz >= 0 && nx < g.dims[0] && ny < g.dims[1] && nz < g.dims[2]) {
                const uint32_t key = morton3((uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
                stt = cs[key];
                ct = ce[key] - stt;
            }
            start[k] = stt;
            cnt[k] = ct;
            L += ct;
        }
        // super-chunk layout of the density/force passes: S chunks, chunk s
        // holds in-cell indices = s mod S of every cell, words laid out in order
        const uint32_t cap = (uint32_t)(kScWords * kWave - 27);
        const uint32_t S = (L + cap - 1) / cap;
        std::vector<uint32_t> &lst = lists[ids[p]];
        uint32_t w0 = 0;
        bool over = S > (uint32_t)kMaxWords;
        std::vector<std::pair<uint32_t, uint32_t>> found;
        for (uint32_t sc = 0; sc < S && !over; ++sc) {
            uint32_t pre[28];
            pre[0] = 0;
            for (int k = 0; k < 27; ++k) {
                const uint32_t c = cnt[k] > sc ? (cnt[k] - sc + S - 1) / S : 0u;
                pre[k + 1] = pre[k] + c;
            }
            const uint32_t size = pre[27];
            const uint32_t nws = (size + kWave - 1) / kWave;
            if (w0 + nws > (uint32_t)kMaxWords) {
                over = true;
                break;
            }
            for (uint32_t q = 0; q < nws; ++q) {
                const uint64_t m = masks[(size_t)(w0 + q) * n + p];
                for (int b = 0; b < 64; ++b) {
                    if (!((m >> b) & 1ull)) continue;
                    const uint32_t v = q * kWave + (uint32_t)b;
                    int k = 0;
                    while (k < 26 && pre[k + 1] <= v) ++k;
                    lst.push_back(ids[start[k] + sc + S * (v - pre[k])]);
                }
            }
            w0 += nws;
        }
        if (over) {
            lst.clear();
            continue;
        }
        std::sort(lst.begin(), lst.end());
    }
    size_t tot = 0;
    const uint32_t m = targets ? nt : n;
    for (uint32_t t = 0; t < m; ++t) {
        const uint32_t i = targets ? targets[t] : t;
        counts[t] = (uint32_t)lists[i].size();
        tot += lists[i].size();
    }
    if (total) *total = tot;
    if (ids_out && tot <= cap) {
        size_t o = 0;
        for (uint32_t t = 0; t < m; ++t)
            for (uint32_t j : lists[targets ? targets[t] : t]) ids_out[o++] = j;
    }
    return st;
}

}  // namespace

extern "C" {

sph_status sph_read_field(sph_ctx *ctx, int field, void *host_dst, size_t bytes)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    return ctx->prec == SPH_FP64 ? read_field_t<double>(ctx, field, host_dst, bytes)
                                 : read_field_t<float>(ctx, field, host_dst, bytes);
}

sph_status sph_debug_neighbors(sph_ctx *ctx, uint32_t *counts, uint32_t *ids, size_t cap, size_t *total)
{
    if (!ctx || (!counts && ctx->n)) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    return ctx->prec == SPH_FP64 ? debug_nbrs_t<double>(ctx, 0, nullptr, counts, ids, cap, total)
                                 : debug_nbrs_t<float>(ctx, 0, nullptr, counts, ids, cap, total);
}

sph_status sph_debug_neighbors_of(sph_ctx *ctx, uint32_t n_targets, const uint32_t *targets, uint32_t *counts,
                                  uint32_t *ids, size_t cap, size_t *total)
{
    if (!ctx || (n_targets && (!targets || !counts))) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    for (uint32_t t = 0; t < n_targets; ++t)
        if (targets[t] >= ctx->n) return SPH_ERR_ARG;
    return ctx->prec == SPH_FP64 ? debug_nbrs_t<double>(ctx, n_targets, targets, counts, ids, cap, total)
                                 : debug_nbrs_t<float>(ctx, n_targets, targets, counts, ids, cap, total);
}

sph_status sph_get_stats(sph_ctx *ctx, uint64_t out[6])
{
    if (!ctx || !out) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    unsigned long long v[6] = {0, 0, 0, 0, 0, 0};
    HIPCHK(ctx, hipMemcpyAsync(v, ctx->stats, sizeof(v), hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int k = 0; k < 6; ++k) out[k] = (uint64_t)v[k];
    return SPH_OK;
}

sph_status sph_get_info(const sph_ctx *ctx, sph_info *info)
{
    if (!ctx || !info) return SPH_ERR_ARG;
    sph_info f{};
    f.n = ctx->n;
    f.n_fluid = ctx->n_fluid;
    f.n_soft = ctx->n_soft;
    f.n_boundary = ctx->n_bnd;
    f.n_body_particles = ctx->nb;
    f.n_kinematic = ctx->nk;
    for (int a = 0; a < 3; ++a) f.grid_dims[a] = (uint32_t)ctx->grid.dims[a];
    f.grid_bits = (uint32_t)ctx->grid.bits;
    f.cell_slots = ctx->grid.nslots;
    f.max_candidates = (uint32_t)(kMaxWords * kWave);   // in cell-aligned words
    f.steps = ctx->steps;
    f.cell_size = ctx->cell_size;
    *info = f;
    return SPH_OK;
}

sph_status sph_profile_begin(sph_ctx *ctx, uint32_t max_steps)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    const size_t need = (size_t)max_steps * kPhases * 2;
    while (ctx->prof_ev.size() < need) {
        hipEvent_t e;
        HIPCHK(ctx, hipEventCreate(&e));
        ctx->prof_ev.push_back(e);
    }
    ctx->prof_phase.assign(need / 2 + 1, 0);
    ctx->prof_used = 0;
    ctx->prof_left = max_steps;
    for (uint32_t k = 0; k < kPhases; ++k) {
        ctx->prof_ms[k] = 0;
        ctx->prof_cnt[k] = 0;
    }
    return SPH_OK;
}

sph_status sph_profile_read(sph_ctx *ctx, double *ms, uint32_t *launches, uint32_t n_phases)
{
    if (!ctx || !ms || !launches) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (size_t k = 0; k + 1 < ctx->prof_used; k += 2) {
        float t = 0;
        HIPCHK(ctx, hipEventElapsedTime(&t, ctx->prof_ev[k], ctx->prof_ev[k + 1]));
        const int ph = ctx->prof_phase[k / 2];
        ctx->prof_ms[ph] += t;
        ctx->prof_cnt[ph] += 1;
    }
    ctx->prof_used = 0;
    ctx->prof_left = 0;
    for (uint32_t k = 0; k < n_phases && k < kPhases; ++k) {
        ms[k] = ctx->prof_ms[k];
        launches[k] = ctx->prof_cnt[k];
    }
    return SPH_OK;
}

sph_status sph_destroy(sph_ctx *ctx)
{
    if (!ctx) return SPH_OK;
    if (!ctx->dead) (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
    delete ctx;
    return SPH_OK;
}

}  // extern "C"
