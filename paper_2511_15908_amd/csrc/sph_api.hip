// C ABI of the SPH hot path (include/sph.h): validation, workspace carving,
// scene upload, the step sequence and host readback.
#include <math.h>
#include <string.h>

#include <algorithm>
#include <limits>
#include <mutex>
#include <type_traits>
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
    uint32_t nb = 0, nk = 0, n_objects = 0, rows = 0, nsprings = 0, K = 1;
    std::vector<int32_t> kin_of_object;   // object -> kinematic index or -1
    std::vector<uint32_t> obj_scene;      // object -> scene of the batch
    std::vector<uint32_t> kin_objects;    // kinematic index -> object
    std::vector<uint8_t> dynamic;         // kinematic index -> free rigid body type (object_kinematic 2)
    std::vector<uint8_t> free_now;        // kinematic index -> currently integrated (not grabbed)
    Grid grid{};                          // scene 0's grid
    double cell_size = 0;
    Phys<float> phf{};                    // scene 0's constants (dt, gravity, v_max are shared)
    Phys<double> phd{};
    uint32_t nscenes = 1, nslots = 0;     // scenes of the batch, key slots of all scenes
    std::vector<Grid> grids;              // per scene, slot0 set
    std::vector<uint32_t> part0;          // first particle id of each scene (+ total)
    void *scene_tab = nullptr;            // device SceneC<T>[nscenes]
    // per-step log of every kinematic / free body
    uint32_t log_cap = 0;
    double *log = nullptr;
    uint32_t *log_count = nullptr;
    uint32_t track_cap = 0;
    double *track = nullptr;
    uint32_t *track_pos = nullptr;
    std::vector<uint8_t> track_on;        // kinematic index -> a track may be active
    // graph replay of two steps
    bool graph_on = false;
    hipGraphExec_t graph_exec = nullptr;
    int graph_parity = 0;
    hipStream_t stream = nullptr;
    // device buffers
    void *pos[2] = {nullptr, nullptr}, *vel[2] = {nullptr, nullptr};
    uint32_t *id[2] = {nullptr, nullptr}, *aux[2] = {nullptr, nullptr};
    int cur = 0;
    Sort sort{};
    uint32_t *inv_perm = nullptr, *cstart = nullptr, *cend = nullptr;
    void *dens = nullptr, *force = nullptr, *fspring = nullptr;
    uint64_t *masks = nullptr;
    uint32_t *row_id = nullptr, *row_ptr = nullptr, *partner = nullptr;
    double *sprm = nullptr;
    uint32_t *slot_id = nullptr, *slot_obj = nullptr;
    double *r_loc = nullptr, *poses = nullptr, *fbody = nullptr, *props = nullptr;
    uint32_t *obj_slot0 = nullptr;
    double *ring = nullptr;
    uint32_t *ring_count = nullptr;
    uint32_t *err = nullptr;
    unsigned long long *stats = nullptr;        // [kStats] sums, filled on request
    unsigned long long *stat_rec = nullptr;     // [nslots][kStatWords] per-slot counters
    int32_t *obj_of_id = nullptr;
    uint32_t max_probes = 0, n_probes = 0;
    double *probe_pts = nullptr, *probe_out = nullptr;
    double *probe_log = nullptr;                 // [log_cap][max_probes] (log and probes both on)
    uint32_t *probe_scene = nullptr;             // [max_probes] scene each probe samples
    int32_t *probe_frame = nullptr;
    std::vector<double> probe_host_pts;
    std::vector<int32_t> probe_host_frame;
    std::vector<uint32_t> probe_host_scene;
    uint64_t steps = 0;
    bool dead = false;
    bool overflowed = false;              // a step exceeded the neighbourhood capacity: state undefined
    int static_dev = -1;                  // device whose static workspace this context holds (sph_init_static)
    std::string last_error;
    std::vector<uint8_t> type_of_id;      // host copy of types (read_field)
    std::vector<sph_params> prms;         // per scene
    // profiling
    uint32_t prof_left = 0;
    uint32_t prof_every = 1;              // events on every k-th armed step
    uint32_t prof_idx = 0;                // armed steps run so far
    bool prof_now = false;                // this step records events
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

// Mass, centre of mass, body-frame inertia about it (and its inverse) of the
// particles of object o; the body frame is that of the initial quaternion.
// False when the inertia tensor is (numerically) singular.
bool body_mass_props(const sph_scene *s, uint32_t o, double *m_out, double com[3], double I[9], double Ii[9])
{
    double m = 0, sx[3] = {0, 0, 0};
    for (uint32_t i = 0; i < s->n; ++i) {
        if (s->type[i] != SPH_BOUNDARY || s->object[i] != (int32_t)o) continue;
        m += s->mass[i];
        for (int a = 0; a < 3; ++a) sx[a] += s->mass[i] * s->x[3 * i + a];
    }
    if (!(m > 0)) return false;
    for (int a = 0; a < 3; ++a) com[a] = sx[a] / m;
    double q[4], R[9];
    quat_normalise(s->object_pose0 + 7 * o + 3, q);
    quat_to_R(q, R);
    for (int a = 0; a < 9; ++a) I[a] = 0;
    for (uint32_t i = 0; i < s->n; ++i) {
        if (s->type[i] != SPH_BOUNDARY || s->object[i] != (int32_t)o) continue;
        const double d[3] = {s->x[3 * i] - com[0], s->x[3 * i + 1] - com[1], s->x[3 * i + 2] - com[2]};
        double r[3];
        for (int a = 0; a < 3; ++a) r[a] = R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2];
        const double rr = r[0] * r[0] + r[1] * r[1] + r[2] * r[2];
        for (int a = 0; a < 3; ++a)
            for (int b = 0; b < 3; ++b) I[3 * a + b] += s->mass[i] * ((a == b ? rr : 0.0) - r[a] * r[b]);
    }
    *m_out = m;
    // inverse by Gauss-Jordan elimination with partial pivoting
    double A[3][6];
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 6; ++b) A[a][b] = b < 3 ? I[3 * a + b] : (b - 3 == a ? 1.0 : 0.0);
    const double scale = fabs(I[0]) + fabs(I[4]) + fabs(I[8]);
    for (int col = 0; col < 3; ++col) {
        int piv = col;
        for (int r = col + 1; r < 3; ++r)
            if (fabs(A[r][col]) > fabs(A[piv][col])) piv = r;
        if (!(fabs(A[piv][col]) > 1e-12 * scale)) return false;
        if (piv != col)
            for (int b = 0; b < 6; ++b) std::swap(A[piv][b], A[col][b]);
        const double d = A[col][col];
        for (int b = 0; b < 6; ++b) A[col][b] /= d;
        for (int r = 0; r < 3; ++r)
            if (r != col) {
                const double f = A[r][col];
                for (int b = 0; b < 6; ++b) A[r][b] -= f * A[col][b];
            }
    }
    for (int a = 0; a < 3; ++a)
        for (int b = 0; b < 3; ++b) Ii[3 * a + b] = A[a][b + 3];
    return true;
}

struct Plan {
    uint32_t n, nb, nk, rows, nsp2, nslots, K, max_probes, nscenes, log_steps, track_steps;
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
    if (p->flags & ~15u) {
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
        if (s->object_kinematic[o] > 2) {
            why = "object_kinematic must be 0 (static), 1 (kinematic) or 2 (free rigid body)";
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
        nk += s->object_kinematic[o] ? 1u : 0u;
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
            if (s->object_kinematic[o] == 2 && (!(s->mass[i] > 0) || !isfinite(s->mass[i]))) {
                why = "particles of a free rigid body need positive finite masses";
                return SPH_ERR_ARG;
            }
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
    for (uint32_t o = 0; o < s->n_objects; ++o) {
        if (s->object_kinematic[o] == 2) {
            double m = 0, com[3], I[9], Ii[9];
            if (!per_obj[o] || !body_mass_props(s, o, &m, com, I, Ii)) {
                why = "a free rigid body needs particles whose inertia tensor is invertible";
                return SPH_ERR_ARG;
            }
        }
    }
    pl.n = n;
    pl.nb = nb;
    pl.nk = nk;
    pl.rows = nsoft;
    pl.nsp2 = 2 * s->n_springs;
    pl.nslots = g.nslots;
    pl.K = p->smoothing_window;
    pl.prec = p->precision;
    pl.max_probes = p->max_probes;
    pl.nscenes = 1;
    pl.log_steps = p->log_steps;
    pl.track_steps = p->track_steps;
    return SPH_OK;
}

// The scenes of a batch concatenated: particle ids, object ids and spring
// ends of scene k follow those of scenes < k.
struct Merged {
    std::vector<double> x, v, mass, pose0, L0, ks, cs;
    std::vector<uint8_t> type, kin;
    std::vector<int32_t> object;
    std::vector<uint32_t> ij;
    std::vector<uint32_t> part0;          // first particle id of each scene, then the total
    sph_scene view{};
};

void merge(const sph_scene *sc, uint32_t ns, Merged &m)
{
    m.part0.assign(1, 0);
    uint32_t obj0 = 0;
    for (uint32_t k = 0; k < ns; ++k) {
        const sph_scene &s = sc[k];
        const uint32_t p0 = m.part0.back();
        m.x.insert(m.x.end(), s.x, s.x + 3 * (size_t)s.n);
        m.v.insert(m.v.end(), s.v, s.v + 3 * (size_t)s.n);
        m.mass.insert(m.mass.end(), s.mass, s.mass + s.n);
        m.type.insert(m.type.end(), s.type, s.type + s.n);
        for (uint32_t i = 0; i < s.n; ++i) m.object.push_back(s.object[i] >= 0 ? s.object[i] + (int32_t)obj0 : -1);
        if (s.n_objects) {
            m.kin.insert(m.kin.end(), s.object_kinematic, s.object_kinematic + s.n_objects);
            m.pose0.insert(m.pose0.end(), s.object_pose0, s.object_pose0 + 7 * (size_t)s.n_objects);
        }
        for (uint32_t e = 0; e < 2 * s.n_springs; ++e) m.ij.push_back(s.spring_ij[e] + p0);
        if (s.n_springs) {
            m.L0.insert(m.L0.end(), s.spring_L0, s.spring_L0 + s.n_springs);
            m.ks.insert(m.ks.end(), s.spring_k, s.spring_k + s.n_springs);
            m.cs.insert(m.cs.end(), s.spring_c, s.spring_c + s.n_springs);
        }
        obj0 += s.n_objects;
        m.part0.push_back(p0 + s.n);
    }
    sph_scene &w = m.view;
    w.n = m.part0.back();
    w.x = m.x.data();
    w.v = m.v.data();
    w.mass = m.mass.data();
    w.type = m.type.data();
    w.object = m.object.data();
    w.n_objects = obj0;
    w.object_kinematic = m.kin.data();
    w.object_pose0 = m.pose0.data();
    w.n_springs = (uint32_t)m.L0.size();
    w.spring_ij = m.ij.data();
    w.spring_L0 = m.L0.data();
    w.spring_k = m.ks.data();
    w.spring_c = m.cs.data();
}

// Validate every scene of a batch with its parameters, the shared settings,
// and the batch totals; grids get their slot0 in the batch's key space.
sph_status validate_batch(const sph_params *p, const sph_scene *sc, uint32_t ns, Plan &pl, std::string &why,
                          std::vector<Grid> *grids, std::vector<double> *csz, Merged *merged)
{
    if (!p || !sc || ns < 1 || ns > 65536u) {
        why = "need 1..65536 scenes with their parameters";
        return SPH_ERR_ARG;
    }
    Plan tot{};
    uint64_t slots = 0, n = 0;
    if (grids) grids->clear();
    if (csz) csz->clear();
    for (uint32_t k = 0; k < ns; ++k) {
        Plan pk{};
        Grid g{};
        double cs = 0;
        const sph_status st = validate(&p[k], &sc[k], pk, why, &g, &cs);
        if (st != SPH_OK) {
            if (ns > 1) why = "scene " + std::to_string(k) + ": " + why;
            return st;
        }
        if (k > 0) {
            const sph_params &a = p[0], &b = p[k];
            if (a.precision != b.precision || a.dt != b.dt || a.v_max != b.v_max ||
                a.smoothing_window != b.smoothing_window || a.log_steps != b.log_steps ||
                a.track_steps != b.track_steps || a.max_probes != b.max_probes ||
                a.gravity[0] != b.gravity[0] || a.gravity[1] != b.gravity[1] || a.gravity[2] != b.gravity[2]) {
                why = "the scenes of a batch share precision, dt, gravity, v_max, smoothing_window, log_steps, "
                      "track_steps, max_probes";
                return SPH_ERR_ARG;
            }
        }
        g.slot0 = (uint32_t)slots;
        slots += g.nslots;
        n += pk.n;
        if (grids) grids->push_back(g);
        if (csz) csz->push_back(cs);
        tot.nb += pk.nb;
        tot.nk += pk.nk;
        tot.rows += pk.rows;
        tot.nsp2 += pk.nsp2;
        tot.max_probes = pk.max_probes;
    }
    if (n > (1u << 24) - 1u || slots > (1u << 30)) {
        why = "batch above 2^24-1 particles or 2^30 cell slots";
        return SPH_ERR_UNSUPPORTED;
    }
    tot.n = (uint32_t)n;
    tot.nslots = (uint32_t)slots;
    tot.K = p[0].smoothing_window;
    tot.prec = p[0].precision;
    tot.nscenes = ns;
    tot.log_steps = p[0].log_steps;
    tot.track_steps = p[0].track_steps;
    if ((uint64_t)tot.track_steps * tot.nk * 128 > (1ull << 36)) {
        why = "track_steps too large";
        return SPH_ERR_ARG;
    }
    pl = tot;
    if (merged) merge(sc, ns, *merged);
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
    c->sort.keys = cv.take<uint32_t>(n * 4);
    c->sort.rank = cv.take<uint32_t>(n * 4);
    c->sort.arrived = cv.take<uint32_t>(n * 4);
    c->sort.counts = cv.take<uint32_t>((size_t)pl.nslots * 4);
    c->sort.tiles = cv.take<uint2>((size_t)cell_scan_tiles(pl.nslots) * 8);
    c->sort.cells = cv.take<uint32_t>((size_t)std::min<uint32_t>(pl.nslots, std::max<uint32_t>(pl.n, 1u)) * 4);
    c->sort.ncell = cv.take<uint32_t>(4);
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
    c->obj_slot0 = cv.take<uint32_t>((size_t)(pl.nk + 1) * 4);
    c->poses = cv.take<double>((size_t)pl.nk * 16 * 8);
    c->props = cv.take<double>((size_t)pl.nk * 24 * 8);
    c->ring = cv.take<double>((size_t)pl.nk * pl.K * 6 * 8);
    c->ring_count = cv.take<uint32_t>((size_t)pl.nk * 4);
    c->err = cv.take<uint32_t>(16);
    c->stats = cv.take<unsigned long long>(8 * 8);
    c->stat_rec = cv.take<unsigned long long>((size_t)pl.nslots * kStatWords * 8);
    c->obj_of_id = cv.take<int32_t>(n * 4);
    c->probe_pts = cv.take<double>((size_t)pl.max_probes * 3 * 8);
    c->probe_frame = cv.take<int32_t>((size_t)pl.max_probes * 4);
    c->probe_out = cv.take<double>((size_t)pl.max_probes * 8);
    c->probe_scene = cv.take<uint32_t>((size_t)pl.max_probes * 4);
    c->probe_log = (pl.log_steps && pl.max_probes && pl.nk)
                       ? cv.take<double>((size_t)pl.log_steps * pl.max_probes * 8)
                       : nullptr;
    c->scene_tab = cv.take<void>((size_t)pl.nscenes * std::max(sizeof(SceneC<float>), sizeof(SceneC<double>)));
    c->log = cv.take<double>((size_t)pl.log_steps * pl.nk * 20 * 8);
    c->log_count = cv.take<uint32_t>((size_t)pl.nk * 4);
    c->track = cv.take<double>((size_t)pl.track_steps * pl.nk * 16 * 8);
    c->track_pos = cv.take<uint32_t>((size_t)pl.nk * 2 * 4);
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
    b.obj_slot0 = c->obj_slot0;
    b.nk = c->nk;
    b.ring = c->ring;
    b.ring_count = c->ring_count;
    b.props = c->props;
    for (int a = 0; a < 3; ++a) b.g[a] = c->prm.gravity[a];
    b.K = c->K;
    b.dt = c->prm.dt;
    b.log = c->log;
    b.log_count = c->log_count;
    b.log_cap = c->log_cap;
    b.track = c->track_cap ? c->track : nullptr;
    b.track_pos = c->track_pos;
    b.track_cap = c->track_cap;
    return b;
}

void prof_mark(sph_ctx *c, int phase, bool begin)
{
    if (!c->prof_now) return;
    if (c->prof_used >= c->prof_ev.size()) return;
    (void)hipEventRecord(c->prof_ev[c->prof_used], c->stream);
    if (begin) c->prof_phase[c->prof_used / 2] = phase;
    ++c->prof_used;
}

template <typename T>
Batch<T> batch(const sph_ctx *c)
{
    return Batch<T>{(const SceneC<T> *)c->scene_tab, c->nscenes, c->nslots};
}

// Neighbour search: keys and per-cell counts, cell table, scatter, reorder
// into the other buffer.
template <typename T>
void neighbour_search(sph_ctx *c)
{
    const uint32_t n = c->n;
    prof_mark(c, 1, true);
    launch_keys<T>(c->stream, n, state<T>(c, c->cur), batch<T>(c), body_args(c), c->sort);
    prof_mark(c, 1, false);
    prof_mark(c, 2, true);
    launch_cell_table(c->stream, c->nslots, c->sort, c->cstart, c->cend);
    launch_cell_scatter(c->stream, n, c->sort, c->cstart);
    prof_mark(c, 2, false);
    prof_mark(c, 3, true);
    launch_reorder<T>(c->stream, n, c->sort, c->cstart, c->cend, state<T>(c, c->cur), state<T>(c, 1 - c->cur),
                      c->inv_perm, (V2<T> *)c->dens, (V4<T> *)c->force);
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
    c->prof_now = c->prof_left && c->prof_idx % c->prof_every == 0u;
    // the kinematic bodies' particles are placed by the key launch (phase "keys")
    neighbour_search<T>(c);
    const State<T> st = state<T>(c, c->cur);
    prof_mark(c, 5, true);
    // the density launch also computes the soft-body springs (phase "density")
    const SpringArgs sa{c->rows, c->row_id, c->row_ptr, c->partner, c->sprm};
    launch_density<T>(s, c->n, st, batch<T>(c), c->cstart, c->cend, (V2<T> *)c->dens, c->masks, c->err, c->stat_rec,
                      c->sort.cells, c->sort.ncell, sa, c->inv_perm, (V4<T> *)c->fspring);
    prof_mark(c, 5, false);
    prof_mark(c, 6, true);
    launch_forces<T>(s, c->n, st, batch<T>(c), c->cstart, c->cend, (const V2<T> *)c->dens, c->masks,
                     (const V4<T> *)c->fspring, (V4<T> *)c->force, c->fbody, c->err, c->stat_rec, c->sort.cells,
                     c->sort.ncell);
    prof_mark(c, 6, false);
    prof_mark(c, 9, true);
    if (c->n_probes) {
        ProbeArgs pa{c->n_probes,  c->probe_pts, c->probe_frame, c->probe_scene, c->poses,
                     c->probe_out, c->probe_log, c->log_count,   c->log_cap,     c->max_probes};
        launch_probe<T>(s, pa, st, batch<T>(c), c->cstart, c->cend);
    }
    prof_mark(c, 9, false);
    // integration and the body wrench share one launch (phase "integrate")
    prof_mark(c, 8, true);
    launch_integrate<T>(s, c->n, st, (const V4<T> *)c->force, phys<T>(c), c->err, ba);
    prof_mark(c, 8, false);
    if (c->prof_left) {
        --c->prof_left;
        ++c->prof_idx;
    }
    c->prof_now = false;
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
    ph.cinv_h64 = kCbrt4 / h;
    ph.alpha6_64 = alpha / 6.0;
    ph.flags = p->flags;
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
    std::vector<uint32_t> slot_id, slot_obj, obj_slot0;
    std::vector<double> r_loc, poses(16 * (size_t)c->nk, 0.0), props(24 * (size_t)c->nk, 0.0);
    std::vector<uint32_t> slot_of(n, 0);
    for (uint32_t k = 0; k < c->nk; ++k) {
        const uint32_t o = c->kin_objects[k];
        double pz[7];
        for (int a = 0; a < 7; ++a) pz[a] = s->object_pose0[7 * o + a];
        if (c->dynamic[k]) {
            // free body: the pose reference point is the particles' centre of mass
            double m = 0, I[9], Ii[9];
            body_mass_props(s, o, &m, pz, I, Ii);
            props[24 * k] = m;
            for (int a = 0; a < 9; ++a) {
                props[24 * k + 1 + a] = I[a];
                props[24 * k + 10 + a] = Ii[a];
            }
            props[24 * k + kPropFree] = 1.0;
        }
        double q[4], R[9];
        quat_normalise(pz + 3, q);
        quat_to_R(q, R);
        for (int a = 0; a < 3; ++a) poses[16 * k + a] = pz[a];
        for (int a = 0; a < 4; ++a) poses[16 * k + 3 + a] = q[a];
        obj_slot0.push_back((uint32_t)slot_id.size());
        for (uint32_t i = 0; i < n; ++i) {
            if (s->type[i] != SPH_BOUNDARY || s->object[i] != (int32_t)o) continue;
            slot_of[i] = (uint32_t)slot_id.size();
            slot_id.push_back(i);
            slot_obj.push_back(k);
            const double d[3] = {s->x[3 * i] - pz[0], s->x[3 * i + 1] - pz[1], s->x[3 * i + 2] - pz[2]};
            for (int a = 0; a < 3; ++a) r_loc.push_back(R[a] * d[0] + R[3 + a] * d[1] + R[6 + a] * d[2]);
        }
    }
    obj_slot0.push_back((uint32_t)slot_id.size());
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
    HIPCHK(c, H2D(c->obj_slot0, obj_slot0.data(), obj_slot0.size() * 4));
    HIPCHK(c, H2D(c->poses, poses.data(), poses.size() * 8));
    HIPCHK(c, H2D(c->props, props.data(), props.size() * 8));
    // zero what must start at zero (fill kernels, no memset nodes)
    launch_clear_u32(st, c->ring_count, c->nk);
    launch_clear_u32(st, c->err, 4);
    launch_clear_u32(st, (uint32_t *)c->stats, 16);
    launch_clear_u32(st, (uint32_t *)c->stat_rec, (size_t)c->nslots * kStatWords * 2);
    launch_clear_u32(st, (uint32_t *)c->dens, (size_t)n * 2 * sizeof(T) / 4);
    launch_clear_u32(st, (uint32_t *)c->force, (size_t)n * 4 * sizeof(T) / 4);
    launch_clear_u32(st, (uint32_t *)c->fspring, (size_t)c->rows * 4 * sizeof(T) / 4);
    launch_clear_u32(st, (uint32_t *)c->fbody, (size_t)c->nb * 6);
    {
        std::vector<SceneC<T>> tab(c->nscenes);
        for (uint32_t k = 0; k < c->nscenes; ++k) {
            tab[k].g = c->grids[k];
            fill_phys(tab[k].ph, &c->prms[k]);
            tab[k].p0 = c->part0[k];
        }
        HIPCHK(c, H2D(c->scene_tab, tab.data(), tab.size() * sizeof(SceneC<T>)));
    }
    launch_clear_u32(st, c->log_count, c->nk);
    launch_clear_u32(st, c->track_pos, 2 * (size_t)c->nk);
    launch_clear_u32(st, c->sort.counts, c->nslots);     // the cell-table scan keeps them zero afterwards
    // first neighbour search, then boundary volumes from the initial configuration
    c->cur = 0;
    if (n) {
        neighbour_search<T>(c);
        launch_psi_obj<T>(st, n, state<T>(c, c->cur), batch<T>(c), c->cstart, c->cend, c->obj_of_id);
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
    if (c->overflowed) return SPH_ERR_CAPACITY;
    if (e) {
        const uint32_t z = 0;
        HIPCHK(c, hipMemcpyAsync(c->err, &z, 4, hipMemcpyHostToDevice, c->stream));
        HIPCHK(c, hipStreamSynchronize(c->stream));
        if (e & ERR_CAPACITY) {
            // the overflowing cells kept stale density and force, which the
            // integration and the wrench then used: the state is no longer a
            // simulation state, so the context refuses further steps
            c->overflowed = true;
            c->last_error = "a cell neighbourhood exceeded the candidate capacity; the state is undefined";
            return SPH_ERR_CAPACITY;
        }
        c->last_error = "non-finite or over-speed particle";
        return SPH_ERR_UNSTABLE;
    }
    return SPH_OK;
}

// Capture two steps (one of each buffer parity) into a graph on the context's stream.
template <typename T>
sph_status capture_two_steps(sph_ctx *c)
{
    hipGraph_t g = nullptr;
    const uint64_t steps = c->steps;
    const uint32_t prof = c->prof_left;
    c->prof_left = 0;
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    c->graph_parity = c->cur;
    one_step<T>(c);
    one_step<T>(c);
    const hipError_t e = hipStreamEndCapture(c->stream, &g);
    c->steps = steps;
    c->prof_left = prof;
    HIPCHK(c, e);
    const hipError_t e2 = hipGraphInstantiate(&c->graph_exec, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    HIPCHK(c, e2);
    return SPH_OK;
}

}  // namespace

// Workspace of sph_init_static: one per device, in the code object's device
// memory, so that a caller that may not allocate device memory can still run
// the whole step.  Host code never uses the array's name as an address: the
// device address comes from hipGetSymbolAddress, once per device.
static __device__ __align__(256) unsigned char scratch[SPH_STATIC_WORKSPACE_BYTES];

namespace {

constexpr int kMaxStaticDevices = 64;
std::mutex g_static_mu;
void *g_static_ptr[kMaxStaticDevices] = {};    // address of `scratch` on each device
bool g_static_busy[kMaxStaticDevices] = {};    // a live context holds that device's array

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

sph_status sph_batch_workspace_size(const sph_params *params, const sph_scene *scenes, uint32_t n_scenes,
                                    size_t *bytes)
{
    if (!bytes) return SPH_ERR_ARG;
    Plan pl{};
    std::string why;
    sph_status st = validate_batch(params, scenes, n_scenes, pl, why, nullptr, nullptr, nullptr);
    if (st != SPH_OK) return st;
    sph_ctx tmp;
    carve(&tmp, pl, nullptr, bytes);
    return SPH_OK;
}

sph_status sph_workspace_size(const sph_params *params, const sph_scene *scene, size_t *bytes)
{
    return sph_batch_workspace_size(params, scene, 1, bytes);
}

sph_status sph_batch_init(const sph_params *params, const sph_scene *scenes, uint32_t n_scenes, void *d_workspace,
                          size_t ws_bytes, void *hip_stream, sph_ctx **out)
{
    if (!out) return SPH_ERR_ARG;
    *out = nullptr;
    Plan pl{};
    std::string why;
    std::vector<Grid> grids;
    std::vector<double> csz;
    Merged mg;
    sph_status st = validate_batch(params, scenes, n_scenes, pl, why, &grids, &csz, &mg);
    if (st != SPH_OK) return st;
    size_t need = 0;
    {
        sph_ctx tmp;
        carve(&tmp, pl, nullptr, &need);
    }
    if (!d_workspace || ws_bytes < need || (reinterpret_cast<uintptr_t>(d_workspace) & 255u)) return SPH_ERR_WORKSPACE;
    sph_ctx *c = new (std::nothrow) sph_ctx();
    if (!c) return SPH_ERR_DEVICE;
    const sph_scene *scene = &mg.view;
    c->prm = params[0];
    c->prms.assign(params, params + n_scenes);
    c->prec = params[0].precision;
    c->n = pl.n;
    c->nb = pl.nb;
    c->nk = pl.nk;
    c->rows = pl.rows;
    c->nsprings = scene->n_springs;
    c->K = pl.K;
    c->n_objects = scene->n_objects;
    c->max_probes = pl.max_probes;
    c->nscenes = n_scenes;
    c->nslots = pl.nslots;
    c->grids = grids;
    c->part0 = mg.part0;
    c->grid = grids[0];
    c->cell_size = csz[0];
    c->log_cap = pl.log_steps;
    c->track_cap = pl.track_steps;
    c->stream = (hipStream_t)hip_stream;
    c->kin_of_object.assign(scene->n_objects, -1);
    for (uint32_t k = 0; k < n_scenes; ++k) c->obj_scene.insert(c->obj_scene.end(), scenes[k].n_objects, k);
    for (uint32_t o = 0; o < scene->n_objects; ++o)
        if (scene->object_kinematic[o]) {
            c->kin_of_object[o] = (int32_t)c->kin_objects.size();
            c->kin_objects.push_back(o);
            c->dynamic.push_back(scene->object_kinematic[o] == 2 ? 1 : 0);
            c->free_now.push_back(scene->object_kinematic[o] == 2 ? 1 : 0);
            c->track_on.push_back(0);
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

sph_status sph_init(const sph_params *params, const sph_scene *scene, void *d_workspace, size_t ws_bytes,
                    void *hip_stream, sph_ctx **out)
{
    return sph_batch_init(params, scene, 1, d_workspace, ws_bytes, hip_stream, out);
}

sph_status sph_init_static(const sph_params *params, const sph_scene *scene, void *hip_stream, sph_ctx **out)
{
    if (!out) return SPH_ERR_ARG;
    *out = nullptr;
    size_t need = 0;
    sph_status st = sph_batch_workspace_size(params, scene, 1, &need);
    if (st != SPH_OK) return st;
    if (need > (size_t)SPH_STATIC_WORKSPACE_BYTES) return SPH_ERR_WORKSPACE;
    int dev = -1;
    if (hipGetDevice(&dev) != hipSuccess) return SPH_ERR_DEVICE;
    if (dev < 0 || dev >= kMaxStaticDevices) return SPH_ERR_UNSUPPORTED;
    void *base = nullptr;
    {
        std::lock_guard<std::mutex> lk(g_static_mu);
        if (g_static_busy[dev]) return SPH_ERR_STATE;
        if (!g_static_ptr[dev]) {
            void *p = nullptr;
            if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return SPH_ERR_DEVICE;
            g_static_ptr[dev] = p;
        }
        base = g_static_ptr[dev];
        g_static_busy[dev] = true;
    }
    st = sph_batch_init(params, scene, 1, base, (size_t)SPH_STATIC_WORKSPACE_BYTES, hip_stream, out);
    if (st != SPH_OK) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[dev] = false;
        return st;
    }
    (*out)->static_dev = dev;
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
    const uint32_t k = (uint32_t)ctx->kin_of_object[object];
    if (ctx->track_on[k]) {
        launch_set_u32x2(ctx->stream, ctx->track_pos + 2 * k, 0u, 0u);
        ctx->track_on[k] = 0;
    }
    launch_set_pose(ctx->stream, ctx->poses + 16 * k, c, qq, v, w);
    HIPCHK(ctx, hipGetLastError());
    return SPH_OK;
}

sph_status sph_set_body_track(sph_ctx *ctx, uint32_t object, uint32_t n, const double *poses)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (object >= ctx->n_objects || ctx->kin_of_object[object] < 0 || n < 1 || n > ctx->track_cap || !poses)
        return SPH_ERR_ARG;
    const uint32_t k = (uint32_t)ctx->kin_of_object[object];
    if (ctx->dynamic[k] && ctx->free_now[k]) {
        ctx->last_error = "a free body moves under its wrench; grab it first";
        return SPH_ERR_ARG;
    }
    std::vector<double> t(16 * (size_t)n, 0.0);
    for (uint32_t e = 0; e < n; ++e) {
        const double *p = poses + 13 * (size_t)e;
        for (int a = 0; a < 13; ++a)
            if (!isfinite(p[a])) return SPH_ERR_ARG;
        const double qn = p[3] * p[3] + p[4] * p[4] + p[5] * p[5] + p[6] * p[6];
        if (!(qn > 0)) return SPH_ERR_ARG;
        double *d = t.data() + 16 * (size_t)e;
        for (int a = 0; a < 13; ++a) d[a] = p[a];
        quat_normalise(p + 3, d + 3);
    }
    double *dst = ctx->track + (size_t)k * ctx->track_cap * 16;
    HIPCHK(ctx, hipMemcpyAsync(dst, t.data(), t.size() * 8, hipMemcpyHostToDevice, ctx->stream));
    launch_set_pose(ctx->stream, ctx->poses + 16 * k, t.data(), t.data() + 3, t.data() + 7, t.data() + 10);
    launch_set_u32x2(ctx->stream, ctx->track_pos + 2 * k, 1u, n);
    ctx->track_on[k] = 1;
    HIPCHK(ctx, hipGetLastError());
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    return SPH_OK;
}

static sph_status set_free(sph_ctx *ctx, uint32_t object, bool free_)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (object >= ctx->n_objects || ctx->kin_of_object[object] < 0) return SPH_ERR_ARG;
    const uint32_t k = (uint32_t)ctx->kin_of_object[object];
    if (!ctx->dynamic[k]) {
        ctx->last_error = "not a free rigid body";
        return SPH_ERR_ARG;
    }
    ctx->free_now[k] = free_ ? 1 : 0;
    if (free_ && ctx->track_on[k]) {
        launch_set_u32x2(ctx->stream, ctx->track_pos + 2 * k, 0u, 0u);
        ctx->track_on[k] = 0;
    }
    launch_set_double(ctx->stream, ctx->props + 24 * k + kPropFree, free_ ? 1.0 : 0.0);
    launch_reset_ring(ctx->stream, ctx->ring_count + k);
    HIPCHK(ctx, hipGetLastError());
    return SPH_OK;
}

sph_status sph_grab_body(sph_ctx *ctx, uint32_t object) { return set_free(ctx, object, false); }
sph_status sph_release_body(sph_ctx *ctx, uint32_t object) { return set_free(ctx, object, true); }

sph_status sph_get_body_state(sph_ctx *ctx, uint32_t object, double c[3], double q[4], double v[3], double w[3])
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (!c || !q || !v || !w || object >= ctx->n_objects || ctx->kin_of_object[object] < 0) return SPH_ERR_ARG;
    double pz[16];
    HIPCHK(ctx, hipMemcpyAsync(pz, ctx->poses + 16 * ctx->kin_of_object[object], sizeof(pz), hipMemcpyDeviceToHost,
                               ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    for (int a = 0; a < 3; ++a) {
        c[a] = pz[a];
        v[a] = pz[7 + a];
        w[a] = pz[10 + a];
    }
    for (int a = 0; a < 4; ++a) q[a] = pz[3 + a];
    return check_err(ctx);
}

sph_status sph_read_log(sph_ctx *ctx, double *out, size_t n_doubles, uint32_t *n_steps)
{
    if (!ctx || !n_steps) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    *n_steps = 0;
    if (!ctx->log_cap || !ctx->nk) return SPH_OK;
    uint32_t cnt = 0;
    HIPCHK(ctx, hipMemcpyAsync(&cnt, ctx->log_count, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const uint32_t m = std::min(cnt, ctx->log_cap);
    const size_t row = (size_t)ctx->nk * 20;
    if (m && (!out || n_doubles < m * row)) return SPH_ERR_ARG;
    // oldest first: ring rows cnt-m .. cnt-1
    const uint32_t first = (cnt - m) % ctx->log_cap;
    const uint32_t a = std::min(m, ctx->log_cap - first);
    if (a)
        HIPCHK(ctx, hipMemcpyAsync(out, ctx->log + first * row, a * row * 8, hipMemcpyDeviceToHost, ctx->stream));
    if (m > a) HIPCHK(ctx, hipMemcpyAsync(out + a * row, ctx->log, (m - a) * row * 8, hipMemcpyDeviceToHost, ctx->stream));
    launch_clear_u32(ctx->stream, ctx->log_count, ctx->nk);
    HIPCHK(ctx, hipGetLastError());
    *n_steps = m;
    return check_err(ctx);
}

sph_status sph_read_probe_log(sph_ctx *ctx, double *out, size_t n_doubles, uint32_t *n_steps)
{
    if (!ctx || !n_steps) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    *n_steps = 0;
    if (!ctx->probe_log || !ctx->n_probes) return SPH_OK;
    uint32_t cnt = 0;
    HIPCHK(ctx, hipMemcpyAsync(&cnt, ctx->log_count, 4, hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    const uint32_t m = std::min(cnt, ctx->log_cap);
    const size_t np = ctx->n_probes, pitch = (size_t)ctx->max_probes * 8;
    if (m && (!out || n_doubles < m * np)) return SPH_ERR_ARG;
    const uint32_t first = (cnt - m) % ctx->log_cap;
    const uint32_t a = std::min(m, ctx->log_cap - first);
    if (a)
        HIPCHK(ctx, hipMemcpy2DAsync(out, np * 8, ctx->probe_log + (size_t)first * ctx->max_probes, pitch, np * 8, a,
                                     hipMemcpyDeviceToHost, ctx->stream));
    if (m > a)
        HIPCHK(ctx, hipMemcpy2DAsync(out + (size_t)a * np, np * 8, ctx->probe_log, pitch, np * 8, m - a,
                                     hipMemcpyDeviceToHost, ctx->stream));
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    *n_steps = m;
    return check_err(ctx);
}

sph_status sph_set_graph(sph_ctx *ctx, int enable)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (ctx->graph_exec) {
        HIPCHK(ctx, hipGraphExecDestroy(ctx->graph_exec));
        ctx->graph_exec = nullptr;
    }
    ctx->graph_on = enable != 0;
    return SPH_OK;
}

sph_status sph_step(sph_ctx *ctx, uint32_t n_steps, void *hip_stream)
{
    if (!ctx) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    if (ctx->overflowed) return SPH_ERR_CAPACITY;
    ctx->stream = (hipStream_t)hip_stream;
    if (!ctx->n) {
        ctx->steps += n_steps;
        return SPH_OK;
    }
    if (ctx->graph_on && !hip_stream) {
        ctx->last_error = "graph replay needs a non-default stream";
        return SPH_ERR_ARG;
    }
    uint32_t k = 0;
    while (k < n_steps) {
        // graph replay: two steps per launch, from the parity the graph was captured at
        if (ctx->graph_on && !ctx->prof_left && n_steps - k >= 2) {
            if (!ctx->graph_exec) {
                const sph_status st =
                    ctx->prec == SPH_FP64 ? capture_two_steps<double>(ctx) : capture_two_steps<float>(ctx);
                if (st != SPH_OK) return st;
            }
            if (ctx->cur == ctx->graph_parity) {
                HIPCHK(ctx, hipGraphLaunch(ctx->graph_exec, ctx->stream));
                ctx->steps += 2;
                k += 2;
                continue;
            }
        }
        if (ctx->prec == SPH_FP64)
            one_step<double>(ctx);
        else
            one_step<float>(ctx);
        ++k;
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
    std::vector<uint32_t> scn(n, 0u);       // world points sample scene 0, body points their body's scene
    for (uint32_t i = 0; i < n; ++i) {
        if (!finite3(points + 3 * i)) return SPH_ERR_ARG;
        if (frame[i] < 0) {
            fr[i] = -1;
        } else {
            if ((uint32_t)frame[i] >= ctx->n_objects || ctx->kin_of_object[frame[i]] < 0) return SPH_ERR_ARG;
            fr[i] = ctx->kin_of_object[frame[i]];
            scn[i] = ctx->obj_scene[frame[i]];
        }
    }
    // the previous upload may still read the host copies
    HIPCHK(ctx, hipStreamSynchronize(ctx->stream));
    if (ctx->graph_exec) {
        HIPCHK(ctx, hipGraphExecDestroy(ctx->graph_exec));
        ctx->graph_exec = nullptr;
    }
    ctx->probe_host_pts.swap(pts);
    ctx->probe_host_frame.swap(fr);
    ctx->probe_host_scene.swap(scn);
    if (n) {
        HIPCHK(ctx, hipMemcpyAsync(ctx->probe_pts, ctx->probe_host_pts.data(), 24 * (size_t)n,
                                   hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(ctx->probe_frame, ctx->probe_host_frame.data(), 4 * (size_t)n,
                                   hipMemcpyHostToDevice, ctx->stream));
        HIPCHK(ctx, hipMemcpyAsync(ctx->probe_scene, ctx->probe_host_scene.data(), 4 * (size_t)n,
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

// Cell slot of every position of the cell order, from the cell table.
std::vector<uint32_t> keys_of_positions(uint32_t n, const std::vector<uint32_t> &cs, const std::vector<uint32_t> &ce)
{
    std::vector<uint32_t> keys(n, 0xffffffffu);
    for (size_t k = 0; k < cs.size(); ++k)
        for (uint32_t p = cs[k]; p < ce[k] && p < n; ++p) keys[p] = (uint32_t)k;
    return keys;
}

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
    std::vector<uint32_t> keys, cs, ce;
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
        cs.resize(c->nslots);
        ce.resize(c->nslots);
        HIPCHK(c, hipMemcpyAsync(cs.data(), c->cstart, cs.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ce.data(), c->cend, ce.size() * 4, hipMemcpyDeviceToHost, s));
    }
    sph_status st = check_err(c);
    if (st == SPH_ERR_DEVICE) return st;
    if (field == SPH_FIELD_KEY) keys = keys_of_positions(n, cs, ce);
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
        case SPH_FIELD_PRESSURE: {
            // the parameters of the particle's own scene
            const uint32_t k =
                (uint32_t)(std::upper_bound(c->part0.begin(), c->part0.end(), i) - c->part0.begin()) - 1u;
            const sph_params &pk = c->prms[k];
            const bool has = !bnd || (pk.flags & SPH_FLAG_UNIFIED_BOUNDARY);
            const double rho = has ? (double)v2[p].x : 0.0;
            double pr = has ? pk.k_pressure * (rho - pk.rho0) : 0.0;
            if ((pk.flags & SPH_FLAG_CLAMP_NEG_PRESSURE) && pr < 0) pr = 0;
            d[i] = field == SPH_FIELD_RHO ? rho : pr;
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
    std::vector<uint32_t> ids(n), aux(n), keys(n), cs(c->nslots), ce(c->nslots);
    std::vector<uint64_t> masks((size_t)kMaxWords * n);
    // positions the step's neighbour passes saw: the reorder's source buffer
    // through the sort permutation (integration has moved the current one)
    std::vector<V4<T>> pos(n), old(n);
    std::vector<uint32_t> old_ids(n), inv(n);
    if (n) {
        HIPCHK(c, hipMemcpyAsync(old.data(), c->pos[1 - c->cur], (size_t)n * sizeof(V4<T>), hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(old_ids.data(), c->id[1 - c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(inv.data(), c->inv_perm, (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ids.data(), c->id[c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(aux.data(), c->aux[c->cur], (size_t)n * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(cs.data(), c->cstart, cs.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(ce.data(), c->cend, ce.size() * 4, hipMemcpyDeviceToHost, s));
        HIPCHK(c, hipMemcpyAsync(masks.data(), c->masks, masks.size() * 8, hipMemcpyDeviceToHost, s));
    }
    sph_status st = check_err(c);
    if (st == SPH_ERR_DEVICE) return st;
    keys = keys_of_positions(n, cs, ce);
    // the reorder moved the particle at old index v to inv_perm[id]
    for (uint32_t v = 0; v < n; ++v) pos[inv[old_ids[v]]] = old[v];
    std::vector<std::vector<uint32_t>> lists(n);
    std::vector<uint8_t> want(n, targets ? 0 : 1);
    if (targets)
        for (uint32_t t = 0; t < nt; ++t) want[targets[t]] = 1;
    for (uint32_t p = 0; p < n; ++p) {
        if (!want[ids[p]]) continue;
        const uint32_t a = aux[p];
        if (aux_type(a) == TY_BOUNDARY && !aux_kin(a)) continue;
        uint32_t sc = 0;
        while (sc + 1 < c->nscenes && c->grids[sc + 1].slot0 <= keys[p]) ++sc;
        const Grid &g = c->grids[sc];
        const uint32_t home = keys[p] - g.slot0;
        // the kernels' candidate filter: within the support of the home cell's box
        T lo[3], hi[3];
        for (int d = 0; d < 3; ++d) {
            lo[d] = std::numeric_limits<T>::infinity();
            hi[d] = -std::numeric_limits<T>::infinity();
        }
        for (uint32_t j = cs[keys[p]]; j < ce[keys[p]]; ++j) {
            const T xyz[3] = {pos[j].x, pos[j].y, pos[j].z};
            for (int d = 0; d < 3; ++d) {
                lo[d] = std::fmin(lo[d], xyz[d]);
                hi[d] = std::fmax(hi[d], xyz[d]);
            }
        }
        const T R2 = std::is_same<T, float>::value ? (T)g.R2_32 : (T)g.R2_64;
        auto near = [&](const V4<T> &q) {
#pragma clang fp contract(off)
            const T dx = std::fmax(std::fmax(lo[0] - q.x, q.x - hi[0]), (T)0);
            const T dy = std::fmax(std::fmax(lo[1] - q.y, q.y - hi[1]), (T)0);
            const T dz = std::fmax(std::fmax(lo[2] - q.z, q.z - hi[2]), (T)0);
            return dx * dx + dy * dy + dz * dz < R2 * (T)1.00390625;
        };
        const int cx = (int)compact3(home), cy = (int)compact3(home >> 1), cz = (int)compact3(home >> 2);
        uint32_t start[27], cnt[27], L = 0;
        for (int k = 0; k < 27; ++k) {
            int ox, oy, oz;
            stencil_offset(k, ox, oy, oz);
            const int nx = cx + ox, ny = cy + oy, nz = cz + oz;
            uint32_t stt = 0, ct = 0;
            if (nx >= 0 && ny >= 0 && nz >= 0 && nx < g.dims[0] && ny < g.dims[1] && nz < g.dims[2]) {
                const uint32_t key = g.slot0 + morton3((uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
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
            std::vector<uint32_t> kept;
            for (uint32_t v = 0; v < size; ++v) {
                int k = 0;
                while (k < 26 && pre[k + 1] <= v) ++k;
                const uint32_t j = start[k] + sc + S * (v - pre[k]);
                if (near(pos[j])) kept.push_back(j);
            }
            // only the words holding culled candidates are written
            const uint32_t nwc = (uint32_t)((kept.size() + kWave - 1) / kWave);
            for (uint32_t q = 0; q < nwc; ++q) {
                const uint64_t m = masks[(size_t)(w0 + q) * n + p];
                for (int b = 0; b < 64; ++b) {
                    if (!((m >> b) & 1ull)) continue;
                    const uint32_t v = q * kWave + (uint32_t)b;
                    if (v < kept.size()) lst.push_back(ids[kept[v]]);
                    else lst.push_back(0xffffffffu);      // a hit past the staged candidates: reported as is
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
    static_assert(kStats == 6, "sph_get_stats reports six counters");
    launch_stats_sum(ctx->stream, ctx->nslots, ctx->stat_rec, ctx->stats);
    HIPCHK(ctx, hipGetLastError());
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
    f.cell_slots = ctx->nslots;
    f.max_candidates = (uint32_t)(kMaxWords * kWave);   // in cell-aligned words
    f.steps = ctx->steps;
    f.cell_size = ctx->cell_size;
    *info = f;
    return SPH_OK;
}

sph_status sph_profile_begin(sph_ctx *ctx, uint32_t max_steps)
{
    return sph_profile_begin_sampled(ctx, max_steps, 1u);
}

sph_status sph_profile_begin_sampled(sph_ctx *ctx, uint32_t max_steps, uint32_t every)
{
    if (!ctx || every < 1u) return SPH_ERR_ARG;
    if (ctx->dead) return SPH_ERR_STATE;
    const size_t need = (size_t)((max_steps + every - 1u) / every) * kPhases * 2;
    while (ctx->prof_ev.size() < need) {
        hipEvent_t e;
        HIPCHK(ctx, hipEventCreate(&e));
        ctx->prof_ev.push_back(e);
    }
    ctx->prof_phase.assign(need / 2 + 1, 0);
    ctx->prof_used = 0;
    ctx->prof_left = max_steps;
    ctx->prof_every = every;
    ctx->prof_idx = 0;
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
    // a static workspace is handed on only after the stream's work on it is done
    if (!ctx->dead || ctx->static_dev >= 0) (void)hipStreamSynchronize(ctx->stream);
    for (hipEvent_t e : ctx->prof_ev) (void)hipEventDestroy(e);
    if (ctx->graph_exec) (void)hipGraphExecDestroy(ctx->graph_exec);
    if (ctx->static_dev >= 0) {
        std::lock_guard<std::mutex> lk(g_static_mu);
        g_static_busy[ctx->static_dev] = false;
    }
    delete ctx;
    return SPH_OK;
}

}  // extern "C"
