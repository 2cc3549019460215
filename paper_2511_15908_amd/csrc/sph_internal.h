// Internal declarations shared by the HIP translation units of libsph.
// Nothing here is part of the C ABI (include/sph.h).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace sphk {

template <typename T>
struct alignas(4 * sizeof(T)) V4 {
    T x, y, z, w;
};
template <typename T>
struct alignas(2 * sizeof(T)) V2 {
    T x, y;
};

// Per-particle state word: bits 0-1 type, bit 2 kinematic body particle,
// bits 8-31 index (spring row of a soft particle, body slot of a kinematic
// boundary particle, object id of a static boundary particle).
enum : uint32_t { TY_FLUID = 0, TY_SOFT = 1, TY_BOUNDARY = 2 };
__host__ __device__ inline uint32_t aux_type(uint32_t a) { return a & 3u; }
__host__ __device__ inline bool aux_kin(uint32_t a) { return (a >> 2) & 1u; }
__host__ __device__ inline uint32_t aux_index(uint32_t a) { return a >> 8; }
__host__ __device__ inline uint32_t aux_make(uint32_t type, bool kin, uint32_t index)
{
    return (type & 3u) | (kin ? 4u : 0u) | (index << 8);
}

// error word bits
enum : uint32_t { ERR_UNSTABLE = 1u, ERR_CAPACITY = 2u };

constexpr int kWave = 64;
#ifndef SPH_SC_WORDS
#define SPH_SC_WORDS 2
#endif
// 64-candidate mask words per super-chunk staged in LDS
constexpr int kScWords = SPH_SC_WORDS;
constexpr int kMaxWords = 64;               // capacity: candidate words per neighbourhood
constexpr int kStats = 6;                   // work counters of a step (see sph_get_stats)
constexpr int kStatWords = 8;               // per-cell-slot counter record, one 64-byte line

// The 27 cells around a home cell: the home cell, then 13 pairs of opposite
// cells, so that a staged super-chunk of candidates holds cells from both
// sides of the home cell.
__host__ __device__ inline void stencil_offset(int k, int &dx, int &dy, int &dz)
{
    const signed char tab[27][3] = {
        {0, 0, 0},
        {1, 0, 0},   {-1, 0, 0},  {0, 1, 0},   {0, -1, 0},  {0, 0, 1},   {0, 0, -1},
        {1, 1, 0},   {-1, -1, 0}, {1, -1, 0},  {-1, 1, 0},  {1, 0, 1},   {-1, 0, -1},
        {1, 0, -1},  {-1, 0, 1},  {0, 1, 1},   {0, -1, -1}, {0, 1, -1},  {0, -1, 1},
        {1, 1, 1},   {-1, -1, -1}, {1, 1, -1}, {-1, -1, 1}, {1, -1, 1},  {-1, 1, -1},
        {-1, 1, 1},  {1, -1, -1}};
    dx = tab[k][0];
    dy = tab[k][1];
    dz = tab[k][2];
}

__host__ __device__ inline uint32_t spread3(uint32_t v)
{
    v &= 0x3ffu;
    v = (v | (v << 16)) & 0x030000FFu;
    v = (v | (v << 8)) & 0x0300F00Fu;
    v = (v | (v << 4)) & 0x030C30C3u;
    v = (v | (v << 2)) & 0x09249249u;
    return v;
}
__host__ __device__ inline uint32_t compact3(uint32_t v)
{
    v &= 0x09249249u;
    v = (v ^ (v >> 2)) & 0x030C30C3u;
    v = (v ^ (v >> 4)) & 0x0300F00Fu;
    v = (v ^ (v >> 8)) & 0xFF0000FFu;
    v = (v ^ (v >> 16)) & 0x000003FFu;
    return v;
}
__host__ __device__ inline uint32_t morton3(uint32_t x, uint32_t y, uint32_t z)
{
    return spread3(x) | (spread3(y) << 1) | (spread3(z) << 2);
}

// Uniform grid constants (by value into kernels).
struct Grid {
    float lo32[3];
    float inv_cs32;
    float R2_32;
    int dims[3];
    int bits;
    uint32_t nslots;   // 2^(3 bits) key slots of this grid
    uint32_t slot0;    // first key of this grid in the batch's key space
    double lo64[3];
    double inv_cs64;
    double R2_64;
};

// Physical constants in the run precision T.
template <typename T>
struct Phys {
    T inv_h;
    T alpha6;     // alpha_3 / 6
    T gc;         // alpha_3 / (2 h^2)
    T gch;        // alpha_3 / (2 h)
    T eps;        // 0.01 h^2
    T two_nu;     // 2 nu
    T gx, gy, gz;
    T dt;
    T vmax2;      // 0: no speed check
    double rho0, kp;
    double inv_h64, alpha6_64;   // FP64 kernel constants of the density sum
    double cinv_h64;             // 4^(1/3) / h
    double psi_scale; // rho0 (for psi init)
    uint32_t flags;
};

// Device pointers of one state buffer (sorted order).
template <typename T>
struct State {
    V4<T> *pos;    // x, y, z, w = mass (fluid/soft) or -psi (boundary)
    V4<T> *vel;    // vx, vy, vz, unused
    uint32_t *id;  // original particle id
    uint32_t *aux; // aux word
};

struct Sort {
    uint32_t *keys;      // [n] cell slot of each particle, current order
    uint32_t *rank;      // [n] arrival rank among the particles of its slot
    uint32_t *arrived;   // [n] current index of the particle at each position of the cell slices
    uint32_t *counts;    // [nslots] particles per slot; zero between steps
    uint2 *tiles;        // [scan tiles] (particles, occupied slots) totals of the slot scan
    uint32_t *cells;     // [min(nslots, n)] occupied slots in slot order
    uint32_t *ncell;     // [1] number of occupied slots
};


// ---- fast math for FP32 terms (1 ulp hardware sqrt / reciprocal); FP64 stays IEEE ----
__device__ __forceinline__ float fsqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
__device__ __forceinline__ double fsqrt(double x) { return sqrt(x); }
__device__ __forceinline__ float frcp(float x) { return __builtin_amdgcn_rcpf(x); }
__device__ __forceinline__ double frcp(double x) { return 1.0 / x; }
__device__ __forceinline__ float frsqrt(float x) { return __builtin_amdgcn_rsqf(x); }
__device__ __forceinline__ double frsqrt(double x) { return 1.0 / sqrt(x); }

// ---- canonical integer decisions shared by every kernel ----

// Canonical cell coordinate: clamp(floor((x - lo) * inv_cs), 0, d - 1), the
// subtraction and the product each rounded in the run precision.
template <typename T>
__device__ __forceinline__ int cell_coord(T x, T lo, T inv, int d)
{
    T t = (x - lo) * inv;
    T f = floor(t);
    if (!(f >= (T)0)) return 0;
    if (f >= (T)d) return d - 1;
    return (int)f;
}

template <typename T>
__device__ __forceinline__ void grid_lo_inv(const Grid &g, T (&lo)[3], T &inv);
template <>
__device__ __forceinline__ void grid_lo_inv<float>(const Grid &g, float (&lo)[3], float &inv)
{
    lo[0] = g.lo32[0];
    lo[1] = g.lo32[1];
    lo[2] = g.lo32[2];
    inv = g.inv_cs32;
}
template <>
__device__ __forceinline__ void grid_lo_inv<double>(const Grid &g, double (&lo)[3], double &inv)
{
    lo[0] = g.lo64[0];
    lo[1] = g.lo64[1];
    lo[2] = g.lo64[2];
    inv = g.inv_cs64;
}

template <typename T>
__device__ __forceinline__ bool within_support(const V4<T> &a, const V4<T> &b, T R2)
{
#pragma clang fp contract(off)
    const T dx = b.x - a.x;
    const T dy = b.y - a.y;
    const T dz = b.z - a.z;
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    return r2 < R2;
}

template <typename T>
__device__ __forceinline__ T grid_R2(const Grid &g);
template <>
__device__ __forceinline__ float grid_R2<float>(const Grid &g) { return g.R2_32; }
template <>
__device__ __forceinline__ double grid_R2<double>(const Grid &g) { return g.R2_64; }


constexpr double kCbrt4 = 1.5874010519681994;   // 4^(1/3), rounded to binary64

// Shape of the cubic spline, (2-q)+^3 - 4 (1-q)+^3 with q = r/h, in FP64 from
// FP64 coordinate differences (exact for FP32 positions).  The density sum
// carries FP64 terms: p = k (rho - rho0) turns a relative density error e
// into e rho / (rho - rho0) (~1e4 e near rest) in the pressure, whose pair
// terms nearly cancel.  The constant alpha/6 multiplies finished sums.
// EXACT = false (FP32 runs): r from an FP32 rsqrt seed and one Newton step in
// FP64, relative error ~5e-15, far below the FP32 result's rounding.
// EXACT = true (FP64 runs): r = sqrt(r^2) in binary64, so the density is good
// to a few ulps and the pressure the force pass sees to ~1e-12 relative.
template <bool EXACT>
__device__ __forceinline__ double spline_r2(double r2, double inv_h, double cinv_h)
{
    double r;
    if constexpr (EXACT) {
        r = sqrt(r2);
    } else {
        const double y = (double)frsqrt(fmaxf((float)r2, 1e-30f));
        r = r2 * y;
        r = fma(0.5 * y, fma(-r, r, r2), r);
    }
    // (2-q)^3 - (c (1-q))+^3 with c^3 = 4; 2 - q is not clamped: the pairs
    // summed pass r^2 < (2h)^2 in T, so 2 - q is at worst a rounding below 0
    const double t2 = fma(-r, inv_h, 2.0);
    const double u = fmax(fma(-r, cinv_h, kCbrt4), 0.0);
    return fma(t2 * t2, t2, -(u * (u * u)));
}

template <bool EXACT>
__device__ __forceinline__ double spline_shape64(double dx, double dy, double dz, double inv_h, double cinv_h)
{
    return spline_r2<EXACT>(fma(dz, dz, fma(dy, dy, dx * dx)), inv_h, cinv_h);
}

// Kernel value W(|c - me|) in FP64 (exact square root in FP64 runs).
template <typename T>
__device__ __forceinline__ double kernel_w64(const V4<T> &c, const V4<T> &me, const Phys<T> &ph)
{
    return ph.alpha6_64 * spline_shape64<sizeof(T) == 8>((double)c.x - (double)me.x, (double)c.y - (double)me.y,
                                                         (double)c.z - (double)me.z, ph.inv_h64, ph.cinv_h64);
}

// --- batches of independent scenes ---
// Every context steps a batch of scenes (one scene is a batch of one).  Each
// scene has its own grid and constants; the key of a particle is the slot0
// of its scene's grid plus its Morton code, so one sort orders the batch
// scene-major and the particles of scene s always occupy the sorted indices
// [p0_s, p0_{s+1}).  Kernels find a work item's scene by binary search.
template <typename T>
struct SceneC {
    Grid g;
    Phys<T> ph;
    uint32_t p0;       // first (sorted) particle index of the scene
    uint32_t pad[3];
};
template <typename T>
struct Batch {
    const SceneC<T> *sc;   // [n] device table
    uint32_t n;            // scenes
    uint32_t nslots;       // key slots of all scenes
};
template <typename T>
__device__ __forceinline__ uint32_t scene_of_particle(const Batch<T> &b, uint32_t i)
{
    uint32_t lo = 0, hi = b.n;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (b.sc[mid].p0 <= i) lo = mid;
        else hi = mid;
    }
    return lo;
}
template <typename T>
__device__ __forceinline__ uint32_t scene_of_slot(const Batch<T> &b, uint32_t k)
{
    uint32_t lo = 0, hi = b.n;
    while (hi - lo > 1u) {
        const uint32_t mid = (lo + hi) >> 1;
        if (b.sc[mid].g.slot0 <= k) lo = mid;
        else hi = mid;
    }
    return lo;
}

// --- launchers (k_grid.hip) ---
struct BodyArgs;
template <typename T>
void launch_keys(hipStream_t s, uint32_t n, State<T> state, const Batch<T> &b, const BodyArgs &ba, Sort &st);
uint32_t cell_scan_tiles(uint32_t nslots);
void launch_cell_table(hipStream_t s, uint32_t nslots, Sort &st, uint32_t *cstart, uint32_t *cend);
void launch_cell_scatter(hipStream_t s, uint32_t n, Sort &st, const uint32_t *cstart);
void launch_clear_u32(hipStream_t s, uint32_t *p, size_t count);
template <typename T>
void launch_reorder(hipStream_t s, uint32_t n, const Sort &st, const uint32_t *cstart, const uint32_t *cend,
                    State<T> in, State<T> out, uint32_t *inv_perm, V2<T> *dens, V4<T> *force);
template <typename T>
void launch_psi_obj(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b, const uint32_t *cstart,
                    const uint32_t *cend, const int32_t *obj_of_id);

// --- launchers (k_sums.hip) ---
// The two neighbour passes run one workgroup per occupied cell (cells, the
// list the cell table wrote, and its length *ncell).
// Soft-body springs (CSR by soft particle), computed by the density launch.
struct SpringArgs {
    uint32_t rows;
    const uint32_t *row_id;   // soft row -> particle id
    const uint32_t *row_ptr;  // [rows+1]
    const uint32_t *partner;  // [2 ns] partner particle id
    const double *prm;        // [3 * 2 ns] L0, k, c per CSR entry
};
template <typename T>
void launch_density(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b,
                    const uint32_t *cstart, const uint32_t *cend, V2<T> *dens, uint64_t *masks,
                    uint32_t *err, unsigned long long *stats, const uint32_t *cells, const uint32_t *ncell,
                    const SpringArgs &sa, const uint32_t *inv_perm, V4<T> *fspring);
template <typename T>
void launch_forces(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b,
                   const uint32_t *cstart, const uint32_t *cend, const V2<T> *dens,
                   const uint64_t *masks, const V4<T> *fspring, V4<T> *force, double *fbody,
                   uint32_t *err, unsigned long long *stats, const uint32_t *cells, const uint32_t *ncell);
// Sum of the per-slot counter records [nslots][kStatWords] into out[kStats].
void launch_stats_sum(hipStream_t s, uint32_t nslots, const unsigned long long *rec, unsigned long long *out);

// --- launchers (k_body.hip) ---
struct BodyArgs {
    uint32_t nb;           // body particles (slots)
    const uint32_t *slot_id;   // slot -> particle id
    const uint32_t *slot_obj;  // slot -> kinematic object index (0..nk-1)
    const double *r_loc;       // [3 nb] body-frame offsets
    double *poses;             // [16 nk]: c[3], q[4], v[3], w[3], pad
    double *fbody;             // [3 nb]
    const uint32_t *obj_slot0; // [nk+1] first body-particle slot of each kinematic object
    uint32_t nk;
    double *ring;              // [nk][K][6]
    uint32_t *ring_count;      // [nk] samples pushed (monotone; reset by sph_reset_smoothing)
    uint32_t K;
    double dt;
    const double *props;       // [24 nk]: mass, I_body[9], I_body^-1[9], free flag (1: integrate), pad
    double g[3];               // gravity (free bodies)
    double *log;               // [log_cap][nk][20]: c, q, v, w, F, T, step (or null)
    uint32_t *log_count;       // [nk] rows written
    uint32_t log_cap;
    const double *track;       // [nk][track_cap][16]: c, q, v, w per step (or null)
    uint32_t *track_pos;       // [2 nk]: next entry, entries
    uint32_t track_cap;
};
constexpr int kPropFree = 19;

// Rotation matrix of a unit quaternion (w, x, y, z), row-major.
__device__ __forceinline__ void quat_R(const double *q, double R[9])
{
#pragma clang fp contract(off)
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

// Placement of kinematic body particle slot s (Sec. 3.2: rigid particles
// keep constant offsets from the parent transform): x = c + R r_loc,
// v = v_c + w x (R r_loc), in binary64, rounded to the run precision; x.w
// (-psi) is kept.
template <typename T>
__device__ __forceinline__ void place_body_particle(const BodyArgs &b, uint32_t s, V4<T> &x, V4<T> &v)
{
#pragma clang fp contract(off)
    const double *pose = b.poses + 16u * b.slot_obj[s];
    double R[9];
    quat_R(pose + 3, R);
    const double r0 = b.r_loc[3 * s], r1 = b.r_loc[3 * s + 1], r2 = b.r_loc[3 * s + 2];
    double rw[3];
    for (int a = 0; a < 3; ++a) rw[a] = R[3 * a] * r0 + R[3 * a + 1] * r1 + R[3 * a + 2] * r2;
    const double *w = pose + 10;
    const double vx = pose[7] + (w[1] * rw[2] - w[2] * rw[1]);
    const double vy = pose[8] + (w[2] * rw[0] - w[0] * rw[2]);
    const double vz = pose[9] + (w[0] * rw[1] - w[1] * rw[0]);
    x.x = (T)(pose[0] + rw[0]);
    x.y = (T)(pose[1] + rw[1]);
    x.z = (T)(pose[2] + rw[2]);
    v = V4<T>{(T)vx, (T)vy, (T)vz, (T)0};
}
void launch_set_pose(hipStream_t s, double *pose_slot, const double c[3], const double q[4],
                     const double v[3], const double w[3]);
void launch_reset_ring(hipStream_t s, uint32_t *ring_count_slot);
void launch_set_double(hipStream_t s, double *slot, double v);
void launch_set_u32x2(hipStream_t s, uint32_t *slot, uint32_t a, uint32_t b);

struct ProbeArgs {
    uint32_t n;
    const double *pts;       // [3n] world or body-frame coordinates
    const int32_t *frame;    // [n] kinematic index of the body frame, or -1
    const uint32_t *scene;   // [n] scene of the batch the probe samples
    const double *poses;     // [16 nk]
    double *out;             // [n]
    double *log;             // [log_cap][stride] per-step copies of out, or null
    const uint32_t *log_row; // the body log's row counter (row of this step)
    uint32_t log_cap, stride;
};
template <typename T>
void launch_probe(hipStream_t s, const ProbeArgs &a, State<T> st, const Batch<T> &b,
                  const uint32_t *cstart, const uint32_t *cend);

template <typename T>
void launch_integrate(hipStream_t s, uint32_t n, State<T> st, const V4<T> *force, const Phys<T> &ph,
                      uint32_t *err, const BodyArgs &b);

}  // namespace sphk
