// Uniform-grid spatial hash of the SPH step (arXiv 2511.15908, Alg. 2: the
// spatial-hash kernels -- cell of each particle, particles per cell,
// cumulative sum, sorted index).  On gfx950 this is a counting sort by cell
// slot: the key kernel counts particles per slot (one atomic per run of equal
// keys in a wavefront; the state is in last step's cell order, so runs are
// long) and keeps each particle's arrival rank; one scan turns the counts
// into the cell start/end table; a scatter places every particle at its
// cell's start plus its rank; the reorder gather puts each cell's particles
// in ascending order of their current index (a rank count over the cell's
// slice: the arrival ranks are not deterministic, this order is), which is
// the order a stable sort by key gives.  The boundary-volume kernel used
// once at init also lives here.
#include "sph_internal.h"

namespace sphk {

// ---------------------------------------------------------------- cell keys

// Key of every particle, its count into counts[key] and its arrival rank
// among the particles of its key.  Lanes of a wavefront hold consecutive
// particles; each run of equal keys takes one atomic for its length, and
// its lanes number themselves from the returned base.
// Kinematic body particles are placed here first (the body's pose of this
// step, Sec. 3.2), so that their keys use the placed positions.
template <typename T>
__global__ __launch_bounds__(256) void k_keys(uint32_t n, State<T> st, Batch<T> b, BodyArgs ba,
                                              uint32_t *__restrict__ keys, uint32_t *__restrict__ rank,
                                              uint32_t *__restrict__ counts)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    const uint32_t lane = threadIdx.x & 63u;
    const bool valid = i < n;          // the valid lanes of a wavefront are a prefix
    uint32_t key = 0xffffffffu;
    if (valid) {
        const Grid g = b.sc[scene_of_particle(b, i)].g;
        T lo[3], inv;
        grid_lo_inv<T>(g, lo, inv);
        V4<T> p = st.pos[i];
        const uint32_t aux = st.aux[i];
        if (aux_type(aux) == TY_BOUNDARY && aux_kin(aux)) {
            V4<T> v;
            place_body_particle<T>(ba, aux_index(aux), p, v);
            st.pos[i] = p;
            st.vel[i] = v;
        }
        const int cx = cell_coord<T>(p.x, lo[0], inv, g.dims[0]);
        const int cy = cell_coord<T>(p.y, lo[1], inv, g.dims[1]);
        const int cz = cell_coord<T>(p.z, lo[2], inv, g.dims[2]);
        key = g.slot0 + morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
        keys[i] = key;
    }
    const uint32_t prev = __shfl_up(key, 1, 64);
    const bool head = valid && (lane == 0u || prev != key);
    const uint64_t heads = __ballot(head);
    const uint64_t upto = lane == 63u ? ~0ull : ((2ull << lane) - 1ull);      // lanes 0 .. lane
    const uint64_t mine = heads & upto;
    const uint32_t hl = mine ? 63u - (uint32_t)__builtin_clzll(mine) : 0u;   // head of this lane's run
    const uint64_t later = heads & ~upto;
    const uint32_t nvalid = (uint32_t)__popcll(__ballot(valid));
    const uint32_t next = later ? (uint32_t)__builtin_ctzll(later) : nvalid;  // head of the next run
    uint32_t base = 0;
    if (head) base = atomicAdd(&counts[key], next - lane);
    base = __shfl(base, (int)hl, 64);
    if (valid) rank[i] = base + (lane - hl);
}

template <typename T>
void launch_keys(hipStream_t s, uint32_t n, State<T> state, const Batch<T> &b, const BodyArgs &ba, Sort &st)
{
    if (!n) return;
    hipLaunchKernelGGL(k_keys<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, state, b, ba, st.keys, st.rank,
                       st.counts);
}
template void launch_keys<float>(hipStream_t, uint32_t, State<float>, const Batch<float> &, const BodyArgs &,
                                 Sort &);
template void launch_keys<double>(hipStream_t, uint32_t, State<double>, const Batch<double> &, const BodyArgs &,
                                  Sort &);

// ---------------------------------------------------------------- cell table
// Exclusive scan of the per-slot counts: cstart[s] = particles in slots
// before s, cend[s] = cstart[s] + counts[s]; at the same time the occupied
// slots are listed in slot order (cells[0 .. *ncell)) and the counts are
// cleared for the next step.  Tiles of kScanTile slots, one 256-thread block
// each (4 slots per thread): a first pass writes the tiles' totals, then
// every block adds up the totals of the tiles before its own (a few hundred
// values at most for the scenes here; above kPrefixTiles tiles one block
// scans the totals in between).  Both scans run on (particles, occupied
// slots) pairs.

constexpr uint32_t kScanThreads = 256, kScanItems = 4, kScanTile = kScanThreads * kScanItems;
constexpr uint32_t kPrefixTiles = 4096;

__device__ __forceinline__ uint2 add2(uint2 a, uint2 b) { return uint2{a.x + b.x, a.y + b.y}; }

// inclusive scan of (x, y) over the block's threads; *total gets the block sum
__device__ __forceinline__ uint2 block_scan_incl(uint2 v, uint2 *wsum, uint2 *total)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    uint2 inc = v;
#pragma unroll
    for (int d = 1; d < 64; d <<= 1) {
        const uint32_t tx = __shfl_up(inc.x, d, 64), ty = __shfl_up(inc.y, d, 64);
        if (lane >= (uint32_t)d) inc = add2(inc, uint2{tx, ty});
    }
    if (lane == 63u) wsum[wv] = inc;
    __syncthreads();
    uint2 before{0u, 0u}, all{0u, 0u};
#pragma unroll
    for (uint32_t w = 0; w < kScanThreads / 64u; ++w) {
        const uint2 x = wsum[w];
        if (w < wv) before = add2(before, x);
        all = add2(all, x);
    }
    *total = all;
    return add2(before, inc);
}

// sum of (x, y) over the block's threads, in thread 0
__device__ __forceinline__ uint2 block_sum(uint2 v, uint2 *wsum)
{
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
#pragma unroll
    for (int d = 32; d >= 1; d >>= 1) v = add2(v, uint2{(uint32_t)__shfl_xor((int)v.x, d, 64),
                                                        (uint32_t)__shfl_xor((int)v.y, d, 64)});
    if (lane == 0u) wsum[wv] = v;
    __syncthreads();
    uint2 all{0u, 0u};
#pragma unroll
    for (uint32_t w = 0; w < kScanThreads / 64u; ++w) all = add2(all, wsum[w]);
    return all;
}

__device__ __forceinline__ uint4 load_counts(const uint32_t *counts, size_t s0, uint32_t nslots, bool &full)
{
    full = s0 + kScanItems <= nslots;        // tiles start 16-byte aligned
    if (full) return *reinterpret_cast<const uint4 *>(counts + s0);
    uint4 c{0u, 0u, 0u, 0u};
    if (s0 < nslots) c.x = counts[s0];
    if (s0 + 1 < nslots) c.y = counts[s0 + 1];
    if (s0 + 2 < nslots) c.z = counts[s0 + 2];
    return c;
}

__device__ __forceinline__ uint2 tile_part(uint4 c)
{
    return uint2{c.x + c.y + c.z + c.w, (uint32_t)(c.x != 0u) + (uint32_t)(c.y != 0u) + (uint32_t)(c.z != 0u) +
                                            (uint32_t)(c.w != 0u)};
}

__global__ __launch_bounds__(kScanThreads) void k_tile_sums(const uint32_t *__restrict__ counts, uint32_t nslots,
                                                            uint2 *__restrict__ tiles)
{
    __shared__ uint2 wsum[kScanThreads / 64];
    bool full;
    const uint4 c = load_counts(counts, (size_t)blockIdx.x * kScanTile + (size_t)threadIdx.x * kScanItems, nslots,
                                full);
    const uint2 all = block_sum(tile_part(c), wsum);
    if (threadIdx.x == 0) tiles[blockIdx.x] = all;
}

// exclusive scan of the ntile tile totals in place (one block; many tiles only)
__global__ __launch_bounds__(kScanThreads) void k_tile_scan(uint2 *__restrict__ tiles, uint32_t ntile)
{
    __shared__ uint2 wsum[kScanThreads / 64];
    uint2 carry{0u, 0u};
    for (uint32_t t0 = 0; t0 < ntile; t0 += kScanThreads) {
        const uint32_t t = t0 + threadIdx.x;
        const uint2 v = t < ntile ? tiles[t] : uint2{0u, 0u};
        uint2 total;
        const uint2 inc = block_scan_incl(v, wsum, &total);
        if (t < ntile) tiles[t] = uint2{carry.x + inc.x - v.x, carry.y + inc.y - v.y};
        carry = add2(carry, total);
        __syncthreads();      // wsum is reused by the next chunk
    }
}

// scanned: tiles hold exclusive prefixes (k_tile_scan ran); otherwise totals
// (block b adds up tiles 0 .. b-1 itself) or nothing (one tile)
__global__ __launch_bounds__(kScanThreads) void k_cell_table(uint32_t *__restrict__ counts, uint32_t nslots,
                                                             const uint2 *__restrict__ tiles, bool scanned,
                                                             uint32_t *__restrict__ cstart,
                                                             uint32_t *__restrict__ cend,
                                                             uint32_t *__restrict__ cells,
                                                             uint32_t *__restrict__ ncell)
{
    __shared__ uint2 wsum[kScanThreads / 64];
    __shared__ uint2 base;
    const uint32_t tid = threadIdx.x;
    if (tiles && !scanned) {
        uint2 v{0u, 0u};
        for (uint32_t t = tid; t < blockIdx.x; t += kScanThreads) v = add2(v, tiles[t]);
        const uint2 all = block_sum(v, wsum);
        if (tid == 0) base = all;
        __syncthreads();
    } else if (tid == 0) {
        base = tiles ? tiles[blockIdx.x] : uint2{0u, 0u};
    }
    const size_t s0 = (size_t)blockIdx.x * kScanTile + (size_t)tid * kScanItems;
    bool full;
    const uint4 c = load_counts(counts, s0, nslots, full);
    const uint2 v = tile_part(c);
    uint2 total;
    const uint2 inc = block_scan_incl(v, wsum, &total);     // synchronises: base is visible
    uint32_t run = inc.x - v.x + base.x, slot = inc.y - v.y + base.y;
    const uint32_t cv[4] = {c.x, c.y, c.z, c.w};
    uint32_t a[4], e[4];
#pragma unroll
    for (uint32_t k = 0; k < 4; ++k) {
        a[k] = run;
        run += cv[k];
        e[k] = run;
        if (cv[k]) cells[slot++] = (uint32_t)(s0 + k);
    }
    if (full) {
        *reinterpret_cast<uint4 *>(cstart + s0) = uint4{a[0], a[1], a[2], a[3]};
        *reinterpret_cast<uint4 *>(cend + s0) = uint4{e[0], e[1], e[2], e[3]};
        *reinterpret_cast<uint4 *>(counts + s0) = uint4{0u, 0u, 0u, 0u};
    } else {
        for (uint32_t k = 0; k < 4; ++k) {
            if (s0 + k >= nslots) break;
            cstart[s0 + k] = a[k];
            cend[s0 + k] = e[k];
            counts[s0 + k] = 0u;
        }
    }
    if (blockIdx.x == gridDim.x - 1u && tid == 0u) *ncell = base.y + total.y;
}

uint32_t cell_scan_tiles(uint32_t nslots) { return (nslots + kScanTile - 1) / kScanTile; }

void launch_cell_table(hipStream_t s, uint32_t nslots, Sort &st, uint32_t *cstart, uint32_t *cend)
{
    const uint32_t nt = cell_scan_tiles(nslots);
    if (!nt) return;
    const bool many = nt > kPrefixTiles;
    if (nt > 1) hipLaunchKernelGGL(k_tile_sums, dim3(nt), dim3(kScanThreads), 0, s, st.counts, nslots, st.tiles);
    if (many) hipLaunchKernelGGL(k_tile_scan, dim3(1), dim3(kScanThreads), 0, s, st.tiles, nt);
    hipLaunchKernelGGL(k_cell_table, dim3(nt), dim3(kScanThreads), 0, s, st.counts, nslots,
                       nt > 1 ? st.tiles : nullptr, many, cstart, cend, st.cells, st.ncell);
}

// ---------------------------------------------------------------- scatter
// Every particle to its cell's start plus its arrival rank.
__global__ __launch_bounds__(256) void k_cell_scatter(uint32_t n, const uint32_t *__restrict__ keys,
                                                      const uint32_t *__restrict__ rank,
                                                      const uint32_t *__restrict__ cstart,
                                                      uint32_t *__restrict__ slot_of)
{
    const uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    slot_of[cstart[keys[i]] + rank[i]] = i;
}

void launch_cell_scatter(hipStream_t s, uint32_t n, Sort &st, const uint32_t *cstart)
{
    if (!n) return;
    hipLaunchKernelGGL(k_cell_scatter, dim3((n + 255) / 256), dim3(256), 0, s, n, st.keys, st.rank, cstart,
                       st.arrived);
}

// ---------------------------------------------------------------- fill

__global__ __launch_bounds__(256) void k_fill_u32(uint32_t *__restrict__ p, size_t count, uint32_t v)
{
    size_t i = (size_t)blockIdx.x * 256u + threadIdx.x;
    const size_t stride = (size_t)gridDim.x * 256u;
    for (; i < count; i += stride) p[i] = v;
}

void launch_clear_u32(hipStream_t s, uint32_t *p, size_t count)
{
    if (!count) return;
    size_t blocks = (count + 255) / 256;
    if (blocks > 4096) blocks = 4096;
    hipLaunchKernelGGL(k_fill_u32, dim3((uint32_t)blocks), dim3(256), 0, s, p, count, 0u);
}

// ---------------------------------------------------------------- reorder

// The particle that arrived at position p of its cell's slice moves to the
// slice start plus the number of the slice's particles with a smaller
// current index: within a cell, ascending current index.  The block's
// positions lie in the cell slices from the first position's cell start to
// the last position's cell end; that range is staged in LDS when it fits
// (cells of ordinary size), otherwise the counts read global memory.  Static
// boundary particles get density and force 0 in their new slot here: the
// neighbour passes never write them (a slot's previous particle may have).
constexpr uint32_t kReorderLds = 2048;

template <typename T>
__global__ __launch_bounds__(256) void k_reorder(uint32_t n, const uint32_t *__restrict__ arrived,
                                                 const uint32_t *__restrict__ keys,
                                                 const uint32_t *__restrict__ cstart,
                                                 const uint32_t *__restrict__ cend, State<T> in, State<T> out,
                                                 uint32_t *__restrict__ inv_perm, V2<T> *__restrict__ dens,
                                                 V4<T> *__restrict__ force)
{
    __shared__ __attribute__((aligned(16))) uint32_t sl[kReorderLds];
    const uint32_t p0 = blockIdx.x * 256u;
    const uint32_t plast = min(p0 + 255u, n - 1u);
    const uint32_t lo = cstart[keys[arrived[p0]]], hi = cend[keys[arrived[plast]]];
    const bool staged = hi - lo <= kReorderLds;        // uniform
    if (staged) {
        for (uint32_t q = lo + threadIdx.x; q < hi; q += 256u) sl[q - lo] = arrived[q];
        __syncthreads();
    }
    const uint32_t p = p0 + threadIdx.x;
    if (p >= n) return;
    const uint32_t j = staged ? sl[p - lo] : arrived[p];
    const uint32_t k = keys[j];
    const uint32_t e0 = cstart[k], e1 = cend[k];
    uint32_t r = 0;
    if (staged) {
        // four slice entries per LDS read in the aligned middle
        uint32_t q = e0 - lo;
        const uint32_t qe = e1 - lo;
        for (; q < qe && (q & 3u); ++q) r += (uint32_t)(sl[q] < j);
        for (; q + 4u <= qe; q += 4u) {
            const uint4 v = *reinterpret_cast<const uint4 *>(&sl[q]);
            r += (uint32_t)(v.x < j) + (uint32_t)(v.y < j) + (uint32_t)(v.z < j) + (uint32_t)(v.w < j);
        }
        for (; q < qe; ++q) r += (uint32_t)(sl[q] < j);
    } else {
        for (uint32_t q = e0; q < e1; ++q) r += (uint32_t)(arrived[q] < j);
    }
    const uint32_t o = e0 + r;
    out.pos[o] = in.pos[j];
    out.vel[o] = in.vel[j];
    const uint32_t id = in.id[j];
    out.id[o] = id;
    const uint32_t aux = in.aux[j];
    out.aux[o] = aux;
    if (aux_type(aux) == TY_BOUNDARY && !aux_kin(aux)) {
        dens[o] = V2<T>{(T)0, (T)0};
        force[o] = V4<T>{(T)0, (T)0, (T)0, (T)0};
    }
    inv_perm[id] = o;
}

template <typename T>
void launch_reorder(hipStream_t s, uint32_t n, const Sort &st, const uint32_t *cstart, const uint32_t *cend,
                    State<T> in, State<T> out, uint32_t *inv_perm, V2<T> *dens, V4<T> *force)
{
    if (!n) return;
    hipLaunchKernelGGL(k_reorder<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, st.arrived, st.keys, cstart, cend,
                       in, out, inv_perm, dens, force);
}
template void launch_reorder<float>(hipStream_t, uint32_t, const Sort &, const uint32_t *, const uint32_t *,
                                    State<float>, State<float>, uint32_t *, V2<float> *, V4<float> *);
template void launch_reorder<double>(hipStream_t, uint32_t, const Sort &, const uint32_t *, const uint32_t *,
                                     State<double>, State<double>, uint32_t *, V2<double> *, V4<double> *);

// ---------------------------------------------------------------- boundary volumes (init only)

// psi_b = rho0 / sum_{k in N(b), same object} W(r_bk), written as pos.w = -psi_b.
template <typename T>
__global__ __launch_bounds__(128) void k_psi(uint32_t n, State<T> st, Batch<T> b,
                                             const uint32_t *__restrict__ cstart,
                                             const uint32_t *__restrict__ cend,
                                             const int32_t *__restrict__ obj_of_id)
{
    uint32_t p = blockIdx.x * 128u + threadIdx.x;
    if (p >= n) return;
    if (aux_type(st.aux[p]) != TY_BOUNDARY) return;
    const SceneC<T> &scn = b.sc[scene_of_particle(b, p)];
    const Grid g = scn.g;
    const Phys<T> ph = scn.ph;
    const V4<T> me = st.pos[p];
    const int32_t ob = obj_of_id[st.id[p]];
    T lo[3], inv;
    grid_lo_inv<T>(g, lo, inv);
    const T R2 = grid_R2<T>(g);
    const int cx = cell_coord<T>(me.x, lo[0], inv, g.dims[0]);
    const int cy = cell_coord<T>(me.y, lo[1], inv, g.dims[1]);
    const int cz = cell_coord<T>(me.z, lo[2], inv, g.dims[2]);
    double acc = 0.0;
    for (int k = 0; k < 27; ++k) {
        int ox, oy, oz;
        stencil_offset(k, ox, oy, oz);
        const int nx = cx + ox, ny = cy + oy, nz = cz + oz;
        if (nx < 0 || ny < 0 || nz < 0 || nx >= g.dims[0] || ny >= g.dims[1] || nz >= g.dims[2]) continue;
        const uint32_t key = g.slot0 + morton3((uint32_t)nx, (uint32_t)ny, (uint32_t)nz);
        const uint32_t e = cend[key];
        for (uint32_t j = cstart[key]; j < e; ++j) {
            if (aux_type(st.aux[j]) != TY_BOUNDARY) continue;
            if (obj_of_id[st.id[j]] != ob) continue;
            const V4<T> c = st.pos[j];
            if (!within_support<T>(me, c, R2)) continue;
            const double dx = (double)c.x - (double)me.x, dy = (double)c.y - (double)me.y;
            const double dz = (double)c.z - (double)me.z;
            const double q = sqrt(dx * dx + dy * dy + dz * dz) * ph.inv_h64;
            const double t2 = fmax(2.0 - q, 0.0);
            const double t1 = fmax(1.0 - q, 0.0);
            acc += ph.alpha6_64 * (t2 * t2 * t2 - 4.0 * (t1 * t1 * t1));
        }
    }
    st.pos[p].w = (T)(-(ph.psi_scale / acc));
}

template <typename T>
static void launch_psi_impl(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b, const uint32_t *cstart,
                            const uint32_t *cend, const int32_t *obj_of_id)
{
    if (!n) return;
    hipLaunchKernelGGL(k_psi<T>, dim3((n + 127) / 128), dim3(128), 0, s, n, st, b, cstart, cend, obj_of_id);
}

}  // namespace sphk

// explicit entry used by the API translation unit
namespace sphk {
template <typename T>
void launch_psi_obj(hipStream_t s, uint32_t n, State<T> st, const Batch<T> &b, const uint32_t *cstart,
                    const uint32_t *cend, const int32_t *obj_of_id)
{
    launch_psi_impl<T>(s, n, st, b, cstart, cend, obj_of_id);
}
template void launch_psi_obj<float>(hipStream_t, uint32_t, State<float>, const Batch<float> &, const uint32_t *,
                                    const uint32_t *, const int32_t *);
template void launch_psi_obj<double>(hipStream_t, uint32_t, State<double>, const Batch<double> &, const uint32_t *,
                                     const uint32_t *, const int32_t *);
}  // namespace sphk
