// SPH neighbour sums of one step (arXiv 2511.15908, Alg. 1): the density /
// pressure pass (Eqs. density, pressure) and the force pass (pressure,
// viscosity and external forces), with fluid/soft <-> boundary-particle
// coupling (Sec. 3.2: every particle type interacts through SPH pressure; the
// rigid particles receive the reaction point forces).
//
// Work decomposition (gfx950, wave64): one workgroup = one wavefront per
// occupied grid cell (cell size 2h, so all neighbours of a particle lie in the
// 27 cells around its own).  Each lane owns one target particle of the home
// cell (two lanes per target when a pass has at most 32 targets, four when it
// has at most 16; each lane then tests and walks every second or fourth
// candidate).  The candidates (particles
// of the 27 cells) are visited in S super-chunks of at
// most kScWords*64: super-chunk s holds every S-th particle of every cell
// (in-cell index = s mod S), which spreads each lane's neighbours evenly over
// the super-chunks.  Candidates farther than the support from the home cell's
// bounding box are culled, the rest staged compacted in LDS; the next
// super-chunk's positions are loaded while the current one is summed.
//  - Density pass: every lane tests every staged candidate (LDS broadcast
//    reads) and keeps one 64-bit hit mask per word in registers; the kernel
//    sum runs over the set bits only, with FP64 terms.  The masks go to HBM.
//  - Force pass: restages the same super-chunks (position, velocity,
//    density) and walks the stored masks, so no pair is tested twice; FP32
//    terms summed per super-chunk, then in FP64.
// The density launch's workgroups past the occupied cells compute the
// soft-body spring forces (two CSR rows each), which the force pass adds.
// No atomics in the sums, so results are bitwise reproducible.
#include <algorithm>

#include "sph_internal.h"

namespace sphk {

// The density pass runs at 5 wavefronts per SIMD (at most 96 VGPRs, a few
// spilled outside the neighbour loop): without the bound the split-pass test
// path takes it to 99 registers and 4 wavefronts, measured 5 % slower.
#ifndef SPH_DENSITY_MIN_WAVES
#define SPH_DENSITY_MIN_WAVES 5
#endif
#define SPH_DENSITY_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SPH_DENSITY_MIN_WAVES)))
// The force pass runs at 6 wavefronts per SIMD (at most 80 VGPRs, a few
// spilled outside the neighbour loop): measured 3 % faster than 5.
#ifndef SPH_FORCES_MIN_WAVES
#define SPH_FORCES_MIN_WAVES 6
#endif
#define SPH_FORCES_OCCUPANCY __attribute__((amdgpu_waves_per_eu(SPH_FORCES_MIN_WAVES)))

struct Nbhd {
    uint32_t start[27];   // first sorted index of each stencil cell
    uint32_t cnt[27];     // particles in each stencil cell
    uint32_t stride;      // S: number of super-chunks
    uint32_t nw;          // candidate words of the neighbourhood
    uint32_t wbase[kMaxWords + 1];  // first word of each super-chunk (S <= kMaxWords)
    uint32_t pre[2][32];  // super-chunks being staged / prefetched (by parity): exclusive
                          // prefix of the per-cell counts, padded
    uint32_t size[2];     // their candidate counts
};

// The neighbour passes launch one workgroup per occupied cell (the cell
// table lists them in slot order: Morton order within a scene, scenes one
// after another); workgroups past the count exit at once.  Blocks are
// dispatched round-robin over the 8 XCDs: within each full group of 512
// cells every XCD gets a run of 64 consecutive cells, so that neighbouring
// cells share its L2; the tail group keeps list order.
#ifndef SPH_XCD_RUN
#define SPH_XCD_RUN 64
#endif
constexpr uint32_t kXcdRun = SPH_XCD_RUN;            // consecutive cells per XCD (power of two)
__device__ __forceinline__ uint32_t list_pos(uint32_t i, uint32_t ncell)
{
    constexpr uint32_t G = 8u * kXcdRun;
    const uint32_t full = ncell - ncell % G;
    if (i >= full) return i;
    const uint32_t grp = i / G, r = i % G;
    return grp * G + (r & 7u) * kXcdRun + (r >> 3);
}

// --- cross-lane moves by DPP (gfx9): row_shr:n reads lane i - n of the same
// 16-lane row, row_bcast:15 / :31 read lane 15 / 31 of the row(s) before
// into the rows enabled by the row mask; a lane with no source keeps `old`.
// Every reduction and scan below needs all 64 lanes active.
constexpr int kShr1 = 0x111, kShr2 = 0x112, kShr4 = 0x114, kShr8 = 0x118, kBc15 = 0x142, kBc31 = 0x143;

template <int CTRL, int ROWS>
__device__ __forceinline__ uint32_t dpp_mov(uint32_t old, uint32_t x)
{
    return (uint32_t)__builtin_amdgcn_update_dpp((int)old, (int)x, CTRL, ROWS, 0xf, false);
}
template <int CTRL, int ROWS>
__device__ __forceinline__ float dpp_mov(float old, float x)
{
    return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(old), __float_as_int(x), CTRL, ROWS, 0xf, false));
}
template <int CTRL, int ROWS>
__device__ __forceinline__ double dpp_mov(double old, double x)
{
    const uint64_t o = (uint64_t)__double_as_longlong(old), v = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)o, (int)(uint32_t)v, CTRL, ROWS, 0xf, false);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_update_dpp((int)(uint32_t)(o >> 32), (int)(uint32_t)(v >> 32), CTRL,
                                                              ROWS, 0xf, false);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

__device__ __forceinline__ uint32_t lane63(uint32_t x) { return (uint32_t)__builtin_amdgcn_readlane((int)x, 63); }
__device__ __forceinline__ float lane63(float x) { return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), 63)); }
__device__ __forceinline__ double lane63(double x)
{
    const uint64_t v = (uint64_t)__double_as_longlong(x);
    const uint32_t lo = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)v, 63);
    const uint32_t hi = (uint32_t)__builtin_amdgcn_readlane((int)(uint32_t)(v >> 32), 63);
    return __longlong_as_double((long long)(((uint64_t)hi << 32) | lo));
}

// Reduction over the 64 lanes, returned to every lane: after the row shifts
// lane 15 of each row holds its row's result; the broadcasts fold rows 0-1
// into lane 31 and then all rows into lane 63.  `id` is op's identity.
template <typename V, typename Op>
__device__ __forceinline__ V wave_reduce(V x, V id, Op op)
{
    x = op(x, dpp_mov<kShr1, 0xf>(id, x));
    x = op(x, dpp_mov<kShr2, 0xf>(id, x));
    x = op(x, dpp_mov<kShr4, 0xf>(id, x));
    x = op(x, dpp_mov<kShr8, 0xf>(id, x));
    x = op(x, dpp_mov<kBc15, 0xa>(id, x));
    x = op(x, dpp_mov<kBc31, 0xc>(id, x));
    return lane63(x);
}

// Inclusive prefix sum over the 64 lanes: row scans, then row 0's total into
// row 1 and row 2's into row 3, then lane 31's total into rows 2-3.
__device__ __forceinline__ uint32_t wave_scan_incl(uint32_t x)
{
    x += dpp_mov<kShr1, 0xf>(0u, x);
    x += dpp_mov<kShr2, 0xf>(0u, x);
    x += dpp_mov<kShr4, 0xf>(0u, x);
    x += dpp_mov<kShr8, 0xf>(0u, x);
    x += dpp_mov<kBc15, 0xa>(0u, x);
    x += dpp_mov<kBc31, 0xc>(0u, x);
    return x;
}

struct OpAdd {
    template <typename V>
    __device__ V operator()(V a, V b) const { return a + b; }
};
struct OpMax {
    __device__ uint32_t operator()(uint32_t a, uint32_t b) const { return max(a, b); }
    __device__ float operator()(float a, float b) const { return fmaxf(a, b); }
    __device__ double operator()(double a, double b) const { return fmax(a, b); }
};
struct OpMin {
    __device__ float operator()(float a, float b) const { return fminf(a, b); }
    __device__ double operator()(double a, double b) const { return fmin(a, b); }
};

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t v) { return wave_reduce(v, 0u, OpAdd{}); }

// Particles of cell k (count c) in super-chunk s of S: ceil((c - s) / S) for
// c > s, taken as floor((c - s - 1 + 1/2) / S) + 1 with invS = 1/S in float.
// A neighbourhood that fits (S <= kMaxWords) has c < 2^13, so (x + 1/2) / S
// lies at least 1/(2 S) >= 1/128 from an integer while the float product is
// off by less than 1e-3: the floor is exact.
__device__ __forceinline__ uint32_t share(uint32_t c, uint32_t s, float invS)
{
    return c > s ? (uint32_t)(((float)(c - s - 1u) + 0.5f) * invS) + 1u : 0u;
}

// Load the 27 cells around `cell` (index in its scene's grid), choose S so every super-chunk fits
// kScWords words, and lay the super-chunks out in words.  Returns false
// (uniformly) when the neighbourhood exceeds kMaxWords words.
__device__ __forceinline__ bool load_nbhd(uint32_t cell, const Grid &g, const uint32_t *__restrict__ cs,
                                          const uint32_t *__restrict__ ce, Nbhd &nb, uint32_t lane)
{
    const int cx = (int)compact3(cell), cy = (int)compact3(cell >> 1), cz = (int)compact3(cell >> 2);
    uint32_t st = 0, cnt = 0;
    if (lane < 27u) {
        int ox, oy, oz;
        stencil_offset((int)lane, ox, oy, oz);
        const int nx = cx + ox, ny = cy + oy, nz = cz + oz;
        if (nx >= 0 && ny >= 0 && nz >= 0 && nx < g.dims[0] && ny < g.dims[1] && nz < g.dims[2]) {
            const uint32_t k = g.slot0 + morton3((uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
            st = cs[k];
            cnt = ce[k] - st;
        }
        nb.start[lane] = st;
        nb.cnt[lane] = cnt;
    }
    const uint32_t L = wave_sum_u32(cnt);
    const uint32_t cap = (uint32_t)(kScWords * kWave - 27);
    const uint32_t S = (L + cap - 1u) / cap;     // >= 1: the home cell is occupied
    if (S > (uint32_t)kMaxWords) return false;
    // words of each super-chunk: lane s < S computes its own size
    const float invS = 1.0f / (float)S;
    uint32_t words = 0;
    for (uint32_t k = 0; k < 27u; ++k) {
        const uint32_t ck = (uint32_t)__builtin_amdgcn_readlane((int)cnt, (int)k);
        words += (lane < S) ? share(ck, lane, invS) : 0u;
    }
    words = (words + (uint32_t)kWave - 1u) / (uint32_t)kWave;
    const uint32_t inc = wave_scan_incl(words);
    if (lane < S) nb.wbase[lane] = inc - words;
    const uint32_t NW = lane63(inc);
    if (lane == 0) {
        nb.stride = S;
        nb.nw = NW;
        nb.wbase[S] = NW;
    }
    __syncthreads();
    return NW <= (uint32_t)kMaxWords;
}

// Prefix of the per-cell shares of super-chunk s into pre[buf] (all lanes
// participate).
__device__ __forceinline__ void begin_chunk(Nbhd &nb, uint32_t s, uint32_t buf, uint32_t lane, float invS)
{
    const uint32_t c = (lane < 27u) ? share(nb.cnt[lane], s, invS) : 0u;
    const uint32_t inc = wave_scan_incl(c);
    if (lane < 32u) nb.pre[buf][lane] = lane < 27u ? inc - c : 0xffffffffu;
    if (lane == 26u) nb.size[buf] = inc;
    __syncthreads();
}

// Sorted indices of the slots v = q*64 + lane of super-chunk s (prefix in
// pre[buf]): cell k = largest with pre[k] <= v, in-cell index s + S (v -
// pre[k]); slots past the super-chunk's size get dflt, and every index is
// kept below n.  The searches of the words run interleaved, so their LDS
// latencies overlap.
__device__ __forceinline__ void chunk_slots(const Nbhd &nb, uint32_t s, uint32_t buf, uint32_t lane, uint32_t dflt,
                                            uint32_t n, uint32_t (&j)[kScWords])
{
    uint32_t k[kScWords];
#pragma unroll
    for (int q = 0; q < kScWords; ++q) k[q] = 0;
#pragma unroll
    for (uint32_t step = 16; step >= 1; step >>= 1) {
#pragma unroll
        for (int q = 0; q < kScWords; ++q)
            if (nb.pre[buf][k[q] + step] <= (uint32_t)q * kWave + lane) k[q] += step;
    }
    const uint32_t sz = nb.size[buf];
#pragma unroll
    for (int q = 0; q < kScWords; ++q) {
        const uint32_t v = (uint32_t)q * kWave + lane;
        j[q] = v < sz ? min(nb.start[k[q]] + s + nb.stride * (v - nb.pre[buf][k[q]]), n - 1u) : dflt;
    }
}

// Bounding box of the home cell's particles (lanes stride over them; the
// same box for every pass over the cell and in both passes of the step).
template <typename T>
__device__ __forceinline__ void cell_box(const V4<T> *__restrict__ pos, uint32_t s0, uint32_t e0, uint32_t lane,
                                         T lo[3], T hi[3])
{
    const T inf = __builtin_huge_val();
    T l0 = inf, l1 = inf, l2 = inf, h0 = -inf, h1 = -inf, h2 = -inf;
    for (uint32_t j = s0 + lane; j < e0; j += kWave) {
        const V4<T> c = pos[j];
        l0 = fmin(l0, c.x);
        l1 = fmin(l1, c.y);
        l2 = fmin(l2, c.z);
        h0 = fmax(h0, c.x);
        h1 = fmax(h1, c.y);
        h2 = fmax(h2, c.z);
    }
    lo[0] = wave_reduce(l0, inf, OpMin{});
    lo[1] = wave_reduce(l1, inf, OpMin{});
    lo[2] = wave_reduce(l2, inf, OpMin{});
    hi[0] = wave_reduce(h0, -inf, OpMax{});
    hi[1] = wave_reduce(h1, -inf, OpMax{});
    hi[2] = wave_reduce(h2, -inf, OpMax{});
}

// A candidate farther than the support from every point of the box cannot
// be a neighbour of any particle in it.  The test is conservative: squared
// distance to the box in T against the squared support enlarged by 2^-8, so
// rounding never drops a pair the canonical predicate accepts.
template <typename T>
__device__ __forceinline__ bool near_box(const V4<T> &c, const T lo[3], const T hi[3], T R2)
{
#pragma clang fp contract(off)
    const T dx = fmax(fmax(lo[0] - c.x, c.x - hi[0]), (T)0);
    const T dy = fmax(fmax(lo[1] - c.y, c.y - hi[1]), (T)0);
    const T dz = fmax(fmax(lo[2] - c.z, c.z - hi[2]), (T)0);
    return dx * dx + dy * dy + dz * dz < R2 * (T)1.00390625;
}

__device__ __forceinline__ uint32_t lanes_below(uint64_t m, uint32_t lane)
{
    return (uint32_t)__popcll(m & ((1ull << lane) - 1ull));
}

// Sign word of r2 - R2 in T for the pair (a, b): its top bit is set exactly
// when the canonical predicate r2 < R2 holds (the difference of two floats
// is zero only when they are equal, and equal values give +0).
template <typename T>
__device__ __forceinline__ uint32_t gap_sign(const V4<T> &a, const V4<T> &b, T R2)
{
#pragma clang fp contract(off)
    const T dx = b.x - a.x;
    const T dy = b.y - a.y;
    const T dz = b.z - a.z;
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const T d = r2 - R2;
    if constexpr (sizeof(T) == 4) return __float_as_uint((float)d);
    else return (uint32_t)((uint64_t)__double_as_longlong((double)d) >> 32);
}

// Hit bits of this lane's particle against nv (<= 32) staged candidates;
// nv is uniform, so empty slots of a super-chunk are never tested.  The
// candidates go from the last to the first, each shifting its sign bit in
// at the bottom (one funnel shift), so candidate b ends at bit b.  They are
// read four at a time before any is tested, so that the four LDS reads are
// in flight together.
constexpr uint32_t kTestBatch = 4;
template <typename T>
__device__ __forceinline__ uint32_t hit_bits(const V4<T> &me, const V4<T> *cand, uint32_t nv, T R2)
{
    uint32_t bits = 0;
    uint32_t b = nv;
    for (; b >= kTestBatch; b -= kTestBatch) {
        V4<T> c[kTestBatch];
#pragma unroll
        for (uint32_t u = 0; u < kTestBatch; ++u) c[u] = cand[b - 1u - u];
#pragma unroll
        for (uint32_t u = 0; u < kTestBatch; ++u)
            bits = __builtin_amdgcn_alignbit(bits, gap_sign<T>(me, c[u], R2), 31u);
    }
    while (b-- > 0u) bits = __builtin_amdgcn_alignbit(bits, gap_sign<T>(me, cand[b], R2), 31u);
    return bits;
}

// One 64-candidate word of hit bits (the first nv slots are candidates).
template <typename T>
__device__ __forceinline__ uint64_t hit_word(const V4<T> &me, const V4<T> *cand, uint32_t nv, T R2)
{
    const uint32_t lo = hit_bits<T>(me, cand, nv < 32u ? nv : 32u, R2);
    const uint32_t hi = nv > 32u ? hit_bits<T>(me, cand + 32, nv - 32u, R2) : 0u;
    return ((uint64_t)hi << 32) | lo;
}

#ifndef SPH_SPLIT_UNROLL
#define SPH_SPLIT_UNROLL 4
#endif

// Split passes (L lanes per target, below): the lane of group g tests only
// the word's candidates g, g + L, g + 2 L, ... (n of them), which are the
// ones it walks; bit i of the result is candidate g + L i.
template <typename T>
__device__ __forceinline__ uint32_t hit_bits_stride(const V4<T> &me, const V4<T> *cand, uint32_t n, uint32_t L, T R2)
{
    uint32_t bits = 0;
#pragma unroll SPH_SPLIT_UNROLL
    for (uint32_t i = n; i-- > 0u;) bits = __builtin_amdgcn_alignbit(bits, gap_sign<T>(me, cand[L * i], R2), 31u);
    return bits;
}

// Bit i of the low 16 bits of x moved to bit 2 i.
__device__ __forceinline__ uint32_t spread16(uint32_t x)
{
    x &= 0xFFFFu;
    x = (x | (x << 8)) & 0x00FF00FFu;
    x = (x | (x << 4)) & 0x0F0F0F0Fu;
    x = (x | (x << 2)) & 0x33333333u;
    x = (x | (x << 1)) & 0x55555555u;
    return x;
}

// Bit i of the low 8 bits of x moved to bit 4 i.
__device__ __forceinline__ uint32_t spread8x4(uint32_t x)
{
    x &= 0xFFu;
    x = (x | (x << 12)) & 0x000F000Fu;
    x = (x | (x << 6)) & 0x03030303u;
    x = (x | (x << 3)) & 0x11111111u;
    return x;
}

// This lane's hit words are held in registers, mw[0] first, and walked
// lowest bit first: the loop over a lane's hits is
//     for (;;) { skip_empty_word(mw, base); if (mw[0] == 0) break;
//                k = base + ctz(mw[0]); clear that bit; ... }
// When the current word is empty the later words move down one place (base
// counts the candidates of the words consumed), so every lane walks its own
// bits without branching on the others.  One move per iteration suffices
// for at most two words: a word only empties by the clearing of its last bit.
static_assert(kScWords >= 1 && kScWords <= 2, "skip_empty_word moves one word per iteration");
__device__ __forceinline__ void skip_empty_word(uint64_t (&mw)[kScWords], int &base)
{
    const bool empty = mw[0] == 0ull;
#pragma unroll
    for (int w = 0; w + 1 < kScWords; ++w) mw[w] = empty ? mw[w + 1] : mw[w];
    mw[kScWords - 1] = empty ? 0ull : mw[kScWords - 1];
    base = empty ? base + kWave : base;
}

// Index of the lowest hit (mw[0] != 0), which is cleared.
__device__ __forceinline__ int take_hit(uint64_t (&mw)[kScWords], int base)
{
    const uint64_t m = mw[0];
    mw[0] = m & (m - 1ull);
    return base + (int)__builtin_ctzll(m);
}

// A staged candidate for the FP64 density terms: position and mass.
struct Cand64 {
    double x, y, z, m;
};
// The term candidates in LDS as two arrays of 16-byte records, (x, y) and
// (z, m): a wavefront's 16-byte reads at scattered slots then spread over
// all LDS banks (32-byte records use every other group of four).
struct CandTerms {
    double2 xy[kScWords * kWave];
    double2 zm[kScWords * kWave];
    template <typename T>
    __device__ __forceinline__ void put(uint32_t k, const V4<T> &c)
    {
        xy[k] = double2{(double)c.x, (double)c.y};
        zm[k] = double2{(double)c.z, (double)fabs(c.w)};
    }
    __device__ __forceinline__ Cand64 get(uint32_t k) const
    {
        const double2 a = xy[k], b = zm[k];
        return Cand64{a.x, a.y, b.x, b.y};
    }
};

// A pass whose cell part holds at most 32 targets (fluid, soft or kinematic
// particles) is served with L = 2 lanes per target, at most 16 with L = 4:
// lanes r, r + 64/L, ... take the r-th target, lane group g = lane / (64/L)
// walking the hit bits of the slots = g mod L, and the L partial sums are
// added at the end of the pass; only group 0 stores.  Divides the neighbour
// loop of cells at walls, at the free surface and in sparse scenes.
struct SplitPass {
    bool split;      // uniform: L > 1
    uint32_t ways;   // uniform: L
    uint32_t grp;    // this lane's group g
    bool lead;       // this lane stores (group 0, or every lane when not split)
    uint64_t bits;   // hit bits this lane walks
};

// Sum of v over the L lanes of this lane's target (fixed order:
// (g0 + g1) + (g2 + g3) for L = 4).
template <typename V>
__device__ __forceinline__ V split_sum(V v, const SplitPass &sp)
{
    if (sp.ways == 4u) v += __shfl_xor(v, 16, 64);
    if (sp.ways >= 2u) v += __shfl_xor(v, 32, 64);
    return v;
}

__device__ __forceinline__ SplitPass split_pass(bool target, bool with_left, uint32_t lane, uint32_t t0, uint32_t e0,
                                               uint32_t s0, const uint32_t *__restrict__ auxv, uint8_t *tmap,
                                               uint32_t &p, bool &act, uint32_t &pc, uint32_t &aux)
{
    const uint64_t tb = __ballot(target);
    const uint32_t nt = (uint32_t)__popcll(tb);
    SplitPass sp{false, 1u, 0u, true, ~0ull};
    if (with_left || nt == 0u || nt > 32u) return sp;
    __syncthreads();                      // the previous pass's readers of tmap are done
    if (target) tmap[lanes_below(tb, lane)] = (uint8_t)lane;
    __syncthreads();
    const uint32_t L = nt <= 16u ? 4u : 2u, shift = L == 4u ? 4u : 5u;
    const uint32_t r = lane & ((kWave / L) - 1u);
    act = r < nt;
    p = act ? t0 + tmap[r] : e0;
    pc = act ? p : s0;
    aux = act ? auxv[pc] : 0u;
    sp.split = true;
    sp.ways = L;
    sp.grp = lane >> shift;
    sp.lead = sp.grp == 0u;
    sp.bits = (L == 4u ? 0x1111111111111111ull : 0x5555555555555555ull) << sp.grp;
    return sp;
}

// ------------------------------------------------------------------ springs

// Spring forces of soft rows r = 2 sb and 2 sb + 1 (mass-spring soft bodies,
// Sec. 3.2), run by workgroups of the density launch past its cells: half a
// wavefront (32 lanes) per row, one spring per lane (rows longer than 32
// loop), the row's sum by a fixed butterfly, so the gathers of a row are in
// flight together.  The force pass reads the result.
template <typename T>
__device__ __forceinline__ void spring_rows(const SpringArgs &a, const uint32_t *__restrict__ inv_perm, State<T> st,
                                            V4<T> *__restrict__ fspring, uint32_t sb)
{
    const uint32_t r = sb * 2u + (threadIdx.x >> 5);
    const uint32_t l = threadIdx.x & 31u;
    const bool row = r < a.rows;
    double f[3] = {0.0, 0.0, 0.0};
    if (row) {
        const uint32_t i = inv_perm[a.row_id[r]];
        const V4<T> xi = st.pos[i], vi = st.vel[i];
        for (uint32_t e = a.row_ptr[r] + l; e < a.row_ptr[r + 1]; e += 32u) {
            const uint32_t j = inv_perm[a.partner[e]];
            const V4<T> xj = st.pos[j], vj = st.vel[j];
            const double d0 = (double)xi.x - (double)xj.x;
            const double d1 = (double)xi.y - (double)xj.y;
            const double d2 = (double)xi.z - (double)xj.z;
            const double len = sqrt(d0 * d0 + d1 * d1 + d2 * d2);
            const double il = 1.0 / len;
            const double e0 = d0 * il, e1 = d1 * il, e2 = d2 * il;
            const double vr = ((double)vi.x - (double)vj.x) * e0 + ((double)vi.y - (double)vj.y) * e1 +
                              ((double)vi.z - (double)vj.z) * e2;
            const double *pr = a.prm + 3u * e;
            const double mag = pr[1] * (len - pr[0]) + pr[2] * vr;
            f[0] -= mag * e0;
            f[1] -= mag * e1;
            f[2] -= mag * e2;
        }
    }
#pragma unroll
    for (int m = 16; m >= 1; m >>= 1) {
        f[0] += __shfl_xor(f[0], m, 32);
        f[1] += __shfl_xor(f[1], m, 32);
        f[2] += __shfl_xor(f[2], m, 32);
    }
    if (row && l == 0) fspring[r] = V4<T>{(T)f[0], (T)f[1], (T)f[2], (T)0};
}

// ------------------------------------------------------------------ density

__device__ __forceinline__ double wave_sum_f64(double v) { return wave_reduce(v, 0.0, OpAdd{}); }

// A cell's particles are served 64 per wavefront pass ("lane mode": lane =
// target).  When a cell holds a little more than a multiple of 64 (common at
// rest: a 2h cell holds exactly 4^3 lattice sites, so slight compression
// tips it over), the last few targets would cost a whole extra pass; they
// are served instead inside the previous pass's super-chunk loop in
// "transposed mode" (lane = candidate, one target at a time, ballot = the
// target's hit word), which costs about 1/20 of a pass per target.
#ifndef SPH_LEFT_DENSITY
#define SPH_LEFT_DENSITY 8
#endif
#ifndef SPH_LEFT_FORCE
#define SPH_LEFT_FORCE 6
#endif
constexpr uint32_t kLeftD = SPH_LEFT_DENSITY;   // most leftover targets of the density pass
constexpr uint32_t kLeftF = SPH_LEFT_FORCE;     // of the force pass

template <typename T>
__global__ __launch_bounds__(64) SPH_DENSITY_OCCUPANCY void k_density(uint32_t n, State<T> st, Batch<T> b,
                                                const uint32_t *__restrict__ cstart,
                                                const uint32_t *__restrict__ cend, V2<T> *__restrict__ dens,
                                                uint64_t *__restrict__ masks, uint32_t *__restrict__ err,
                                                unsigned long long *__restrict__ stats,
                                                const uint32_t *__restrict__ cells,
                                                const uint32_t *__restrict__ n_occupied, SpringArgs sa,
                                                const uint32_t *__restrict__ inv_perm, V4<T> *__restrict__ fspring)
{
    __shared__ Nbhd nb;
    __shared__ V4<T> cand[kScWords * kWave];         // tests: T positions, inf past the end
    __shared__ CandTerms cand64;                 // terms: FP64 positions and masses
    __shared__ double accl[kLeftD > 0 ? kLeftD : 1];
    __shared__ unsigned long long cstat[5];
    __shared__ uint8_t tmap[kWave];
    constexpr bool kExact = sizeof(T) == 8;          // FP64 runs: binary64 square root in the terms
    const uint32_t lane = threadIdx.x;
    const uint32_t ncq = *n_occupied;
    if (blockIdx.x >= ncq) {
        // the workgroups past the occupied cells: two spring rows each
        const uint32_t sb = blockIdx.x - ncq;
        if (sb < (sa.rows + 1u) / 2u) spring_rows<T>(sa, inv_perm, st, fspring, sb);
        return;
    }
    const uint32_t slot = cells[list_pos(blockIdx.x, ncq)];
    const uint32_t s0 = cstart[slot], e0 = cend[slot];
    if (s0 >= e0) return;
    const SceneC<T> &scn = b.sc[scene_of_slot(b, slot)];
    const Grid g = scn.g;
    const Phys<T> ph = scn.ph;
    // unified boundary reading: boundary particles have a density of their own
    const bool unified = (ph.flags & 8u) != 0u;
    if (!load_nbhd(slot - g.slot0, g, cstart, cend, nb, lane)) {
        if (lane == 0) atomicOr(err, ERR_CAPACITY);
        return;
    }
    const uint32_t S = nb.stride;
    const float invS = 1.0f / (float)S;
    const T R2 = grid_R2<T>(g);
    const T inf = __builtin_huge_val();
    T blo[3], bhi[3];
    cell_box<T>(st.pos, s0, e0, lane, blo, bhi);
    const uint32_t ncell = e0 - s0, rem = ncell % kWave;
    const bool use_left = ncell > (uint32_t)kWave && rem != 0u && rem <= kLeftD;
    const uint32_t nlane = use_left ? ncell / kWave : (ncell + kWave - 1) / kWave;
    const uint32_t nleft = use_left ? rem : 0u;
    const uint32_t left0 = s0 + kWave * nlane;
    // work counters of the cell (uniform), added to the slot's own record
    // (kept in LDS by lane 0 rather than in registers)
    if (lane < 5u) cstat[lane] = 0ull;
    for (uint32_t ch = 0; ch < nlane; ++ch) {
        const uint32_t t0 = s0 + kWave * ch;
        const bool with_left = (ch + 1 == nlane) && nleft;
        uint32_t p = t0 + lane;
        bool act = p < e0;
        uint32_t pc = act ? p : s0;
        uint32_t aux = act ? st.aux[pc] : 0u;
        // a pass with at most 32 targets is split: two or four lanes per
        // target (no lane then serves the cell's static boundary particles,
        // whose density and force the reorder has already set to 0)
        const SplitPass sp = split_pass(act && (aux_type(aux) != TY_BOUNDARY || aux_kin(aux) || unified), with_left,
                                        lane, t0, e0, s0, st.aux, tmap, p, act, pc, aux);
        V4<T> me = st.pos[pc];
        me.x = act ? me.x : inf;
        me.y = act ? me.y : inf;
        me.z = act ? me.z : inf;
        const double mx = (double)me.x, my = (double)me.y, mz = (double)me.z;
        const bool fs = act && aux_type(aux) != TY_BOUNDARY;
        const bool dn = fs || (act && unified);        // lanes whose density is summed
        const bool want = act && (dn || aux_kin(aux));
        const bool lanes_any = __ballot(want) != 0ull;
        if (!lanes_any && !with_left) continue;
        if (with_left && lane < nleft) accl[lane] = 0.0;
        double acc = 0.0;
        uint32_t npair = 0, witer = 0, ncand = 0, nleftpair_d = 0, nleftpair_f = 0;
        // the candidates of super-chunk sc + 1 are loaded while sc is summed
        V4<T> nxt[kScWords];
        {
            uint32_t j[kScWords];
            begin_chunk(nb, 0u, 0u, lane, invS);
            chunk_slots(nb, 0u, 0u, lane, s0, n, j);
#pragma unroll
            for (int q = 0; q < kScWords; ++q) nxt[q] = st.pos[j[q]];
        }
        for (uint32_t sc = 0; sc < S; ++sc) {
            const uint32_t buf = sc & 1u;
            const uint32_t csize = nb.size[buf];
            V4<T> cur[kScWords];
#pragma unroll
            for (int q = 0; q < kScWords; ++q) cur[q] = nxt[q];
            if (sc + 1u < S) {
                uint32_t j[kScWords];
                begin_chunk(nb, sc + 1u, buf ^ 1u, lane, invS);
                chunk_slots(nb, sc + 1u, buf ^ 1u, lane, s0, n, j);
#pragma unroll
                for (int q = 0; q < kScWords; ++q) nxt[q] = st.pos[j[q]];
            }
            // stage the super-chunk's candidates near the cell's box, compacted
            uint32_t size = 0;
#pragma unroll
            for (int q = 0; q < kScWords; ++q) {
                const uint32_t v = q * kWave + lane;
                const bool in = v < csize;
                const V4<T> c = cur[q];
                const bool keep = in && near_box<T>(c, blo, bhi, R2);
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const uint32_t slot_c = size + lanes_below(km, lane);
                    cand[slot_c] = c;
                    cand64.put(slot_c, c);
                }
                size += (uint32_t)__popcll(km);
            }
#pragma unroll
            for (int q = 0; q < kScWords; ++q) {
                const uint32_t v = q * kWave + lane;
                if (v >= size) cand[v] = V4<T>{inf, inf, inf, (T)0};
            }
            ncand += size;
            __syncthreads();
            // the super-chunk owns words [w0, w0 + its pre-culling words); only the
            // first nwc hold candidates after culling and are written and read
            const uint32_t nwc = (size + (uint32_t)kWave - 1u) / (uint32_t)kWave;
            const uint32_t w0 = nb.wbase[sc];
            if (lanes_any) {
                uint64_t mw[kScWords];
#pragma unroll
                for (int q = 0; q < kScWords; ++q) {
                    uint64_t m = 0;
                    if ((uint32_t)q < nwc) {
                        const uint32_t nv = size > (uint32_t)q * kWave ? min(size - (uint32_t)q * kWave, (uint32_t)kWave) : 0u;
                        if (sp.split) {
                            // each group tests the candidates it walks; the full word
                            // (stored for the force pass) joins the groups.  Slots past
                            // the word's nv hold +inf (no hit) up to slot 63.
                            const uint32_t L = sp.ways, g = sp.grp, nl = (nv + L - 1u) / L;
                            const uint32_t bits = hit_bits_stride<T>(me, cand + q * kWave + g, nl, L, R2);
                            // candidate g + L i at bit g + L i (the spread bits stay below
                            // bit 32 - L + 1, so the shift by g keeps each word apart)
                            uint32_t lo, hi;
                            if (L == 4u) {
                                lo = spread8x4(bits) << g;
                                hi = spread8x4(bits >> 8) << g;
                                lo |= (uint32_t)__shfl_xor((int)lo, 16, 64);
                                hi |= (uint32_t)__shfl_xor((int)hi, 16, 64);
                            } else {
                                lo = spread16(bits) << g;
                                hi = spread16(bits >> 16) << g;
                            }
                            lo |= (uint32_t)__shfl_xor((int)lo, 32, 64);
                            hi |= (uint32_t)__shfl_xor((int)hi, 32, 64);
                            m = ((uint64_t)hi << 32) | lo;
                        } else {
                            m = hit_word<T>(me, cand + q * kWave, nv, R2);
                        }
                        if (act && sp.lead) masks[(size_t)(w0 + q) * n + p] = m;
                        npair += (want && sp.lead) ? (uint32_t)__popcll(m) : 0u;
                    }
                    mw[q] = dn ? (m & sp.bits) : 0ull;
                }
                {
                    uint32_t mine = 0;
#pragma unroll
                    for (int q = 0; q < kScWords; ++q) mine += (uint32_t)__popcll(mw[q]);
                    witer += wave_reduce(mine, 0u, OpMax{});
                }
                // kernel sum over this lane's neighbours among the staged
                // candidates, in units of alpha/6
                if (size <= (uint32_t)kWave) {
                    // one word holds the whole (culled) super-chunk: no word moves
                    uint64_t m = mw[0];
                    while (m) {
                        const int k = (int)__builtin_ctzll(m);
                        m &= m - 1ull;
                        const Cand64 c = cand64.get(k);
                        acc = fma(c.m, spline_shape64<kExact>(c.x - mx, c.y - my, c.z - mz, ph.inv_h64, ph.cinv_h64),
                                  acc);
                    }
                } else {
                    int base = 0;
                    for (;;) {
                        skip_empty_word(mw, base);
                        if (mw[0] == 0ull) break;
                        const int k = take_hit(mw, base);
                        const Cand64 c = cand64.get(k);
                        acc = fma(c.m, spline_shape64<kExact>(c.x - mx, c.y - my, c.z - mz, ph.inv_h64, ph.cinv_h64),
                                  acc);
                    }
                }
            }
            if (with_left) {
                // transposed mode: lane = staged candidate slot
                for (uint32_t t = 0; t < nleft; ++t) {
                    const uint32_t pt = left0 + t;
                    const uint32_t at = st.aux[pt];
                    const bool fs_t = aux_type(at) != TY_BOUNDARY;
                    const bool dn_t = fs_t || unified;
                    if (!dn_t && !aux_kin(at)) continue;    // uniform: static boundary
                    const V4<T> mt = st.pos[pt];
                    const double tx = (double)mt.x, ty = (double)mt.y, tz = (double)mt.z;
                    double part = 0.0;
#pragma unroll
                    for (int q = 0; q < kScWords; ++q) {
                        if ((uint32_t)q < nwc) {
                            const V4<T> c = cand[q * kWave + lane];   // far past the chunk end
                            const bool hit = within_support<T>(mt, c, R2);
                            const uint64_t m = __ballot(hit);
                            if (lane == 0) masks[(size_t)(w0 + q) * n + pt] = m;
                            const uint32_t cnt = (uint32_t)__popcll(m);
                            nleftpair_f += cnt;
                            nleftpair_d += dn_t ? cnt : 0u;
                            if (dn_t && hit) {
                                const Cand64 c64 = cand64.get(q * kWave + lane);
                                part = fma(c64.m,
                                           spline_shape64<kExact>(c64.x - tx, c64.y - ty, c64.z - tz, ph.inv_h64,
                                                                  ph.cinv_h64),
                                           part);
                            }
                        }
                    }
                    part = wave_sum_f64(part);
                    if (lane == 0) accl[t] += part;
                }
            }
            __syncthreads();
        }
        {
            // step statistics: neighbour pairs of density targets, of force
            // targets, candidate tests, wavefronts, loop iterations
            uint32_t nd = dn ? npair : 0u, nf = npair;
            nd = wave_sum_u32(nd);
            nf = wave_sum_u32(nf);
            if (lane == 0) {
                cstat[0] += nd + nleftpair_d;
                cstat[1] += nf + nleftpair_f;
                cstat[2] += (unsigned long long)ncand * (kWave + nleft);
                cstat[3] += 1u;
                cstat[4] += witer;
            }
        }
        if (sp.split) acc = split_sum(acc, sp);
        if (act && sp.lead) {
            V2<T> d{(T)0, (T)0};
            if (dn) {
                const double rho = ph.alpha6_64 * acc;
                double pr = ph.kp * (rho - ph.rho0);
                if ((ph.flags & 1u) && pr < 0.0) pr = 0.0;
                d.x = (T)rho;
                d.y = (T)(pr / (rho * rho));
            }
            dens[p] = d;
        }
        if (with_left && lane < nleft) {
            const uint32_t pt = left0 + lane;
            const bool dn_t = aux_type(st.aux[pt]) != TY_BOUNDARY || unified;
            V2<T> d{(T)0, (T)0};
            if (dn_t) {
                const double rho = ph.alpha6_64 * accl[lane];
                double pr = ph.kp * (rho - ph.rho0);
                if ((ph.flags & 1u) && pr < 0.0) pr = 0.0;
                d.x = (T)rho;
                d.y = (T)(pr / (rho * rho));
            }
            dens[pt] = d;
        }
    }
    __syncthreads();
    if (lane < 5u) stats[(size_t)slot * kStatWords + lane] += cstat[lane];
}

// ------------------------------------------------------------------ forces

// Pair force on particle a from particle c (both terms of Alg. 1's force
// pass), accumulated into f.  gradW_ac = g(r) x_ac with
//   g = (dW/dr)/r = alpha/(2 h^2) (4 t1^2 - t2^2) / q,  t1 = (1-q)+, t2 = (2-q)+.
// 4 t1^2 - t2^2 = (2 t1 - t2)(2 t1 + t2) = -min(q, 2-q) max(4-3q, 2-q) on
// 0 <= q <= 2 (q < 1: -q (4-3q); q >= 1: -(2-q)^2), so -g is
//   alpha/(2h) min(q, 2-q) max(4-3q, 2-q) / r,
// finite and 0 at r = 0 (self pair).  A boundary particle takes the pressure
// and density of its fluid/soft partner (pressure mirroring), its mass is
// psi_b; two boundary particles exert nothing.  Every scalar factor is
// symmetric in (a, c), so the pressure force c computes on itself from a is
// the exact IEEE negation.  The viscosity term sv (v_a - v_c) is summed as
// -sv v_c here plus v_a times the sum of sv (fw), added once per chunk: two
// operations fewer per pair, with the pair antisymmetric up to rounding.
// P_mir is the pressure a boundary partner takes from this particle: P_a,
// or 0 with the single-boundary-term flag.  KIN = false: particle a is not a
// boundary particle; PLAIN: neither boundary flag (2, 4) is set.  With the
// unified reading (flag 8) a boundary particle keeps its own density and
// pressure: its staged mirror factor cv.w is 0 and a boundary target does not
// take its partner's values either (mirror = false).
// The velocities mv and cv come multiplied by 4 nu (vel_scaled), the uniform
// factor of the viscosity term.
template <typename T>
__device__ __forceinline__ V4<T> vel_scaled(V4<T> v, const Phys<T> &ph)
{
    // both sides of a pair scale alike, so v_a - v_c stays antisymmetric
    const T k = ph.two_nu * (T)2;
    v.x *= k;
    v.y *= k;
    v.z *= k;
    return v;
}

template <typename T, bool KIN, bool PLAIN>
__device__ __forceinline__ void pair_force(const V4<T> &me, const V4<T> &mv, T rho_a, T P_a, T P_mir, bool isBa,
                                           bool mirror, T ma, const V4<T> &c, const V4<T> &cv, const V2<T> &cd,
                                           const Phys<T> &ph, T &fx, T &fy, T &fz, T &fw)
{
    const T dx = me.x - c.x, dy = me.y - c.y, dz = me.z - c.z;
    const T r2 = fma(dz, dz, fma(dy, dy, dx * dx));
    const T rs = frsqrt(max(r2, (T)1e-30));      // 1/r
    const T q = (r2 * rs) * ph.inv_h;
    const T t2 = (T)2 - q;
    const T gn = (min(q, t2) * max(fma((T)-3, q, (T)4), t2)) * (ph.gch * rs);   // -g
    // cv.w is 1 for a mirrored boundary candidate (0 otherwise), whose staged
    // density and pressure term are 0: the mirrored values enter by one FMA
    // each; boundary candidates carry -psi_b in c.w
    const bool isBc = c.w < (T)0;
    const T mc = fabs(c.w);
    const T Pc = fma(cv.w, P_mir, cd.y);
    const T rc = fma(cv.w, rho_a, cd.x);
    T Pa = P_a, ra = rho_a;
    if (KIN) {
        const T Pb = (!PLAIN && (ph.flags & 2u)) ? (T)0 : cd.y;
        Pa = (isBa && mirror) ? Pb : P_a;
        ra = (isBa && mirror) ? cd.x : rho_a;
    }
    const T mg = (ma * mc) * gn;                   // -m_a m_c g
    // pressure: -m_a m_c (P_a/rho_a^2 + P_c/rho_c^2) g
    T sp = (Pa + Pc) * mg;
    // viscosity: 2 nu m_a m_c [2/(rho_a+rho_c)] g r^2/(r^2+eps), one
    // reciprocal, with the 4 nu on the velocities
    T sv = -((mg * r2) * frcp((ra + rc) * (r2 + ph.eps)));
    if (KIN) {
        const bool bb = isBa && isBc;
        sp = bb ? (T)0 : sp;
        sv = bb ? (T)0 : sv;
    }
    if (!PLAIN) {
        const bool novisc = (ph.flags & 4u) && (isBa || isBc);
        sv = novisc ? (T)0 : sv;
    }
    fx = fma(sp, dx, fma(-sv, cv.x, fx));
    fy = fma(sp, dy, fma(-sv, cv.y, fy));
    fz = fma(sp, dz, fma(-sv, cv.z, fz));
    fw += sv;
}

// Pair forces of one lane's hits among the staged candidates (walking its
// hit words).  KIN = false when no lane of the wavefront serves a kinematic
// boundary particle: the target-side pressure mirroring then drops out.
// ONE: the staged super-chunk fits one word (no word moves).
template <typename T, bool KIN, bool PLAIN, bool ONE>
__device__ __forceinline__ void walk_forces(uint64_t (&mw)[kScWords], const V4<T> &me, const V4<T> &mv,
                                            const V2<T> &md, T P_mir, bool kin, bool mirror, T ma, const V4<T> *cp,
                                            const V4<T> *cvel, const V2<T> *cden, const Phys<T> &ph, T &cx, T &cy,
                                            T &cz, T &cw)
{
    if (ONE) {
        uint64_t m = mw[0];
        while (m) {
            const int k = (int)__builtin_ctzll(m);
            m &= m - 1ull;
            pair_force<T, KIN, PLAIN>(me, mv, md.x, md.y, P_mir, kin, mirror, ma, cp[k], cvel[k], cden[k], ph, cx, cy,
                                      cz, cw);
        }
        return;
    }
    int base = 0;
    for (;;) {
        skip_empty_word(mw, base);
        if (mw[0] == 0ull) break;
        const int k = take_hit(mw, base);
        pair_force<T, KIN, PLAIN>(me, mv, md.x, md.y, P_mir, kin, mirror, ma, cp[k], cvel[k], cden[k], ph, cx, cy, cz,
                                  cw);
    }
}

// Force on a lane-mode or transposed-mode target from its accumulated pair
// sum: fluid/soft add gravity and springs; kinematic boundary particles keep
// the reaction for the body wrench.
template <typename T>
__device__ __forceinline__ void store_force(uint32_t p, uint32_t aux, T ma, double fx, double fy, double fz,
                                            const Phys<T> &ph, const V4<T> *__restrict__ fspring,
                                            V4<T> *__restrict__ force, double *__restrict__ fbody)
{
    if (aux_type(aux) != TY_BOUNDARY) {
        double ex = ma * ph.gx, ey = ma * ph.gy, ez = ma * ph.gz;
        if (aux_type(aux) == TY_SOFT) {
            const V4<T> sp = fspring[aux_index(aux)];
            ex += sp.x;
            ey += sp.y;
            ez += sp.z;
        }
        force[p] = V4<T>{(T)(fx + ex), (T)(fy + ey), (T)(fz + ez), (T)0};
    } else if (aux_kin(aux)) {
        force[p] = V4<T>{(T)fx, (T)fy, (T)fz, (T)0};
        double *fb = fbody + 3u * aux_index(aux);
        fb[0] = fx;
        fb[1] = fy;
        fb[2] = fz;
    }
}

template <typename T>
__global__ __launch_bounds__(64) SPH_FORCES_OCCUPANCY void k_forces(uint32_t n, State<T> st, Batch<T> b,
                                               const uint32_t *__restrict__ cstart,
                                               const uint32_t *__restrict__ cend, const V2<T> *__restrict__ dens,
                                               const uint64_t *__restrict__ masks,
                                               const V4<T> *__restrict__ fspring, V4<T> *__restrict__ force,
                                               double *__restrict__ fbody, unsigned long long *__restrict__ stats,
                                               const uint32_t *__restrict__ cells,
                                               const uint32_t *__restrict__ n_occupied)
{
    __shared__ Nbhd nb;
    __shared__ V4<T> cp[kScWords * kWave];
    __shared__ V4<T> cvel[kScWords * kWave];
    __shared__ V2<T> cden[kScWords * kWave];
    __shared__ double accf[kLeftF > 0 ? kLeftF : 1][3];
    __shared__ unsigned long long cstat;   // neighbour-loop iterations of the cell
    __shared__ uint8_t tmap[kWave];
    const uint32_t lane = threadIdx.x;
    const uint32_t ncq = *n_occupied;
    if (blockIdx.x >= ncq) return;
    const uint32_t slot = cells[list_pos(blockIdx.x, ncq)];
    const uint32_t s0 = cstart[slot], e0 = cend[slot];
    if (s0 >= e0) return;
    const SceneC<T> &scn = b.sc[scene_of_slot(b, slot)];
    const Grid g = scn.g;
    const Phys<T> ph = scn.ph;
    const bool mirror = (ph.flags & 8u) == 0u;    // pressure mirroring (not the unified reading)
    if (!load_nbhd(slot - g.slot0, g, cstart, cend, nb, lane)) return;   // flagged by the density pass
    const uint32_t S = nb.stride;
    const float invS = 1.0f / (float)S;
    const T R2 = grid_R2<T>(g);
    T blo[3], bhi[3];
    cell_box<T>(st.pos, s0, e0, lane, blo, bhi);
    const uint32_t ncell = e0 - s0, rem = ncell % kWave;
    const bool use_left = ncell > (uint32_t)kWave && rem != 0u && rem <= kLeftF;
    const uint32_t nlane = use_left ? ncell / kWave : (ncell + kWave - 1) / kWave;
    const uint32_t nleft = use_left ? rem : 0u;
    const uint32_t left0 = s0 + kWave * nlane;
    if (lane == 0) cstat = 0ull;
    for (uint32_t ch = 0; ch < nlane; ++ch) {
        const uint32_t t0 = s0 + kWave * ch;
        const bool with_left = (ch + 1 == nlane) && nleft;
        uint32_t p = t0 + lane;
        bool act = p < e0;
        uint32_t pc = act ? p : s0;
        uint32_t aux = act ? st.aux[pc] : 0u;
        const SplitPass sp = split_pass(act && (aux_type(aux) != TY_BOUNDARY || aux_kin(aux)), with_left, lane,
                                        t0, e0, s0, st.aux, tmap, p, act, pc, aux);
        const V4<T> me = st.pos[pc];
        const V4<T> mv = vel_scaled(st.vel[pc], ph);
        const V2<T> md = dens[pc];
        const bool fs = act && aux_type(aux) != TY_BOUNDARY;
        const bool kin = act && aux_kin(aux);
        const bool tgt = fs || kin;
        const bool lanes_any = __ballot(tgt) != 0ull;
        const bool wave_kin = __ballot(kin) != 0ull;
        if (!lanes_any && !with_left) continue;
        if (with_left && lane < 3u * nleft) accf[lane / 3u][lane % 3u] = 0.0;
        const T ma = fabs(me.w);
        double fx = 0.0, fy = 0.0, fz = 0.0;
        uint32_t witer = 0;
        // the positions of super-chunk sc + 1 are loaded while sc is summed
        V4<T> nxt[kScWords];
        uint32_t nj[kScWords];
        begin_chunk(nb, 0u, 0u, lane, invS);
        chunk_slots(nb, 0u, 0u, lane, s0, n, nj);
#pragma unroll
        for (int q = 0; q < kScWords; ++q) nxt[q] = st.pos[nj[q]];
        for (uint32_t sc = 0; sc < S; ++sc) {
            const uint32_t buf = sc & 1u;
            const uint32_t csize = nb.size[buf];
            V4<T> cur[kScWords];
            uint32_t cj[kScWords];
#pragma unroll
            for (int q = 0; q < kScWords; ++q) {
                cur[q] = nxt[q];
                cj[q] = nj[q];
            }
            if (sc + 1u < S) {
                begin_chunk(nb, sc + 1u, buf ^ 1u, lane, invS);
                chunk_slots(nb, sc + 1u, buf ^ 1u, lane, s0, n, nj);
#pragma unroll
                for (int q = 0; q < kScWords; ++q) nxt[q] = st.pos[nj[q]];
            }
            // the density pass's compacted layout: candidates near the cell's
            // box in chunk order (slots past it are never hit)
            uint32_t size = 0;
#pragma unroll
            for (int q = 0; q < kScWords; ++q) {
                const uint32_t v = q * kWave + lane;
                const bool in = v < csize;
                const uint32_t j = cj[q];
                const V4<T> c = cur[q];
                const bool keep = in && near_box<T>(c, blo, bhi, R2);
                const uint64_t km = __ballot(keep);
                if (keep) {
                    const uint32_t o = size + lanes_below(km, lane);
                    cp[o] = c;
                    V4<T> cv = vel_scaled(st.vel[j], ph);
                    cv.w = (mirror && c.w < (T)0) ? (T)1 : (T)0;    // mirror factor for the pair loop
                    cvel[o] = cv;
                    cden[o] = dens[j];
                }
                size += (uint32_t)__popcll(km);
            }
            // the super-chunk owns words [w0, w0 + its pre-culling words); only the
            // first nwc hold candidates after culling and are written and read
            const uint32_t nwc = (size + (uint32_t)kWave - 1u) / (uint32_t)kWave;
            const uint32_t w0 = nb.wbase[sc];
            uint64_t mw[kScWords];
#pragma unroll
            for (int q = 0; q < kScWords; ++q) {
                uint64_t m = 0;
                if ((uint32_t)q < nwc && tgt) m = masks[(size_t)(w0 + q) * n + p];
                mw[q] = m & sp.bits;
            }
            __syncthreads();
            if (lanes_any) {
                {
                    uint32_t mine = 0;
#pragma unroll
                    for (int q = 0; q < kScWords; ++q) mine += (uint32_t)__popcll(mw[q]);
                    witer += wave_reduce(mine, 0u, OpMax{});
                }
                // a super-chunk holds ~1/S of the neighbours: sum it in T, then in FP64
                T cx = (T)0, cy = (T)0, cz = (T)0, cw = (T)0;
                const T P_mir = (ph.flags & 2u) ? (T)0 : md.y;
                const bool one = size <= (uint32_t)kWave;
                if (wave_kin || (ph.flags & 6u)) {
                    if (one)
                        walk_forces<T, true, false, true>(mw, me, mv, md, P_mir, kin, mirror, ma, cp, cvel, cden, ph,
                                                          cx, cy, cz, cw);
                    else
                        walk_forces<T, true, false, false>(mw, me, mv, md, P_mir, kin, mirror, ma, cp, cvel, cden, ph,
                                                           cx, cy, cz, cw);
                } else {
                    if (one)
                        walk_forces<T, false, true, true>(mw, me, mv, md, P_mir, kin, mirror, ma, cp, cvel, cden, ph,
                                                          cx, cy, cz, cw);
                    else
                        walk_forces<T, false, true, false>(mw, me, mv, md, P_mir, kin, mirror, ma, cp, cvel, cden, ph,
                                                           cx, cy, cz, cw);
                }
                // the viscosity terms' target velocity, once per chunk
                cx = fma(mv.x, cw, cx);
                cy = fma(mv.y, cw, cy);
                cz = fma(mv.z, cw, cz);
                fx += (double)cx;
                fy += (double)cy;
                fz += (double)cz;
            }
            if (with_left) {
                // transposed mode: lane = staged candidate slot
                for (uint32_t t = 0; t < nleft; ++t) {
                    const uint32_t pt = left0 + t;
                    const uint32_t at = st.aux[pt];
                    const bool kin_t = aux_kin(at);
                    if (aux_type(at) == TY_BOUNDARY && !kin_t) continue;   // uniform: static boundary
                    const V4<T> mt = st.pos[pt];
                    const V4<T> mvt = vel_scaled(st.vel[pt], ph);
                    const V2<T> mdt = dens[pt];
                    T cx = (T)0, cy = (T)0, cz = (T)0, cw = (T)0;
#pragma unroll
                    for (int q = 0; q < kScWords; ++q) {
                        if ((uint32_t)q < nwc) {
                            const uint64_t m = masks[(size_t)(w0 + q) * n + pt];
                            const uint32_t v = q * kWave + lane;
                            if ((m >> lane) & 1ull)
                                pair_force<T, true, false>(mt, mvt, mdt.x, mdt.y, (ph.flags & 2u) ? (T)0 : mdt.y,
                                                           kin_t, mirror, fabs(mt.w), cp[v], cvel[v], cden[v], ph,
                                                           cx, cy, cz, cw);
                        }
                    }
                    cx = fma(mvt.x, cw, cx);
                    cy = fma(mvt.y, cw, cy);
                    cz = fma(mvt.z, cw, cz);
                    cx = wave_reduce(cx, (T)0, OpAdd{});
                    cy = wave_reduce(cy, (T)0, OpAdd{});
                    cz = wave_reduce(cz, (T)0, OpAdd{});
                    if (lane == 0) {
                        accf[t][0] += (double)cx;
                        accf[t][1] += (double)cy;
                        accf[t][2] += (double)cz;
                    }
                }
            }
            __syncthreads();
        }
        if (lane == 0) cstat += witer;
        if (sp.split) {
            fx = split_sum(fx, sp);
            fy = split_sum(fy, sp);
            fz = split_sum(fz, sp);
        }
        if (tgt && sp.lead) store_force<T>(p, aux, ma, fx, fy, fz, ph, fspring, force, fbody);
        if (with_left && lane < nleft) {
            const uint32_t pt = left0 + lane;
            const uint32_t at = st.aux[pt];
            if (aux_type(at) != TY_BOUNDARY || aux_kin(at))
                store_force<T>(pt, at, fabs(st.pos[pt].w), accf[lane][0], accf[lane][1], accf[lane][2], ph, fspring,
                               force, fbody);
        }
    }
    __syncthreads();
    if (lane == 0) stats[(size_t)slot * kStatWords + 5] += cstat;
}

// Work counters: each cell slot's record is only touched by the one
// workgroup that serves the slot in a launch, so the sums need no atomics;
// this reduction (one block per counter, fixed order) adds them up on demand.
__global__ __launch_bounds__(256) void k_stats_sum(uint32_t nslots, const unsigned long long *__restrict__ rec,
                                                   unsigned long long *__restrict__ out)
{
    __shared__ unsigned long long part[256];
    const uint32_t k = blockIdx.x, t = threadIdx.x;
    unsigned long long v = 0;
    for (uint32_t i = t; i < nslots; i += 256u) v += rec[(size_t)i * kStatWords + k];
    part[t] = v;
    __syncthreads();
    for (uint32_t h = 128; h >= 1; h >>= 1) {
        if (t < h) part[t] += part[t + h];
        __syncthreads();
    }
    if (t == 0) out[k] = part[0];
}

void launch_stats_sum(hipStream_t s, uint32_t nslots, const unsigned long long *rec, unsigned long long *out)
{
    hipLaunchKernelGGL(k_stats_sum, dim3(kStats), dim3(256), 0, s, nslots, rec, out);
}

// One workgroup per occupied cell at most: min(particles, slots).
inline uint32_t cell_grid(uint32_t n, uint32_t nslots) { return std::max(1u, std::min(n, nslots)); }

template <typename T>
void launch_density(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b, const uint32_t *cstart,
                    const uint32_t *cend, V2<T> *dens, uint64_t *masks, uint32_t *err, unsigned long long *stats,
                    const uint32_t *cells, const uint32_t *ncell, const SpringArgs &sa, const uint32_t *inv_perm,
                    V4<T> *fspring)
{
    if (!n) return;
    // the occupied cells first (at most cell_grid of them), then the spring rows
    const uint32_t grid = cell_grid(n, b.nslots) + (sa.rows + 1u) / 2u;
    hipLaunchKernelGGL(k_density<T>, dim3(grid), dim3(64), 0, s, n, st, b, cstart, cend, dens, masks, err, stats,
                       cells, ncell, sa, inv_perm, fspring);
}

template <typename T>
void launch_forces(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b, const uint32_t *cstart,
                   const uint32_t *cend, const V2<T> *dens, const uint64_t *masks, const V4<T> *fspring,
                   V4<T> *force, double *fbody, uint32_t *err, unsigned long long *stats, const uint32_t *cells,
                   const uint32_t *ncell)
{
    (void)err;
    if (!n) return;
    hipLaunchKernelGGL(k_forces<T>, dim3(cell_grid(n, b.nslots)), dim3(64), 0, s, n, st, b, cstart, cend, dens,
                       masks, fspring, force, fbody, stats, cells, ncell);
}

template void launch_density<float>(hipStream_t, uint32_t, State<float>, const Batch<float> &, const uint32_t *,
                                    const uint32_t *, V2<float> *, uint64_t *, uint32_t *, unsigned long long *,
                                    const uint32_t *, const uint32_t *, const SpringArgs &, const uint32_t *,
                                    V4<float> *);
template void launch_density<double>(hipStream_t, uint32_t, State<double>, const Batch<double> &, const uint32_t *,
                                     const uint32_t *, V2<double> *, uint64_t *, uint32_t *, unsigned long long *,
                                     const uint32_t *, const uint32_t *, const SpringArgs &, const uint32_t *,
                                     V4<double> *);
template void launch_forces<float>(hipStream_t, uint32_t, State<float>, const Batch<float> &, const uint32_t *,
                                   const uint32_t *, const V2<float> *, const uint64_t *, const V4<float> *,
                                   V4<float> *, double *, uint32_t *, unsigned long long *, const uint32_t *,
                                   const uint32_t *);
template void launch_forces<double>(hipStream_t, uint32_t, State<double>, const Batch<double> &, const uint32_t *,
                                    const uint32_t *, const V2<double> *, const uint64_t *, const V4<double> *,
                                    V4<double> *, double *, uint32_t *, unsigned long long *, const uint32_t *,
                                    const uint32_t *);

}  // namespace sphk
