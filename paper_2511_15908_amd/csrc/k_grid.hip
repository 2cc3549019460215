// Uniform-grid spatial hash of the SPH step (arXiv 2511.15908, Alg. 2: the
// four "spatial hash" kernels -- cell of each particle, particles per cell,
// cumulative sum, sorted index).  On gfx950 the count/scan/scatter sequence
// is a stable LSD radix sort of Morton cell keys (8-bit digits), followed by
// one gather that reorders the particle state into cell order and writes the
// cell start/end table.  The boundary-volume kernel used once at init also
// lives here.
#include "sph_internal.h"

namespace sphk {

// ---------------------------------------------------------------- cell keys

template <typename T>
__global__ __launch_bounds__(256) void k_keys(uint32_t n, const V4<T> *__restrict__ pos, Batch<T> b,
                                              uint32_t *__restrict__ keys)
{
    uint32_t i = blockIdx.x * 256u + threadIdx.x;
    if (i >= n) return;
    const Grid g = b.sc[scene_of_particle(b, i)].g;
    T lo[3], inv;
    grid_lo_inv<T>(g, lo, inv);
    V4<T> p = pos[i];
    int cx = cell_coord<T>(p.x, lo[0], inv, g.dims[0]);
    int cy = cell_coord<T>(p.y, lo[1], inv, g.dims[1]);
    int cz = cell_coord<T>(p.z, lo[2], inv, g.dims[2]);
    keys[i] = g.slot0 + morton3((uint32_t)cx, (uint32_t)cy, (uint32_t)cz);
}

template <typename T>
void launch_keys(hipStream_t s, uint32_t n, const V4<T> *pos, const Batch<T> &b, uint32_t *keys)
{
    if (!n) return;
    hipLaunchKernelGGL(k_keys<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, pos, b, keys);
}
template void launch_keys<float>(hipStream_t, uint32_t, const V4<float> *, const Batch<float> &, uint32_t *);
template void launch_keys<double>(hipStream_t, uint32_t, const V4<double> *, const Batch<double> &, uint32_t *);

// ---------------------------------------------------------------- radix sort
// Tile of 2048 keys per block (256 threads x 8 rounds).  hist is digit-major:
// hist[d * nblk + b] = count of digit d in block b; the per-digit scan turns
// it into the offset of block b within digit d and puts the digit's total in
// dbase[d]; the scatter adds the exclusive scan of the totals.

constexpr int RS_THREADS = 256;
constexpr int RS_ROUNDS = 8;
constexpr int RS_TILE = RS_THREADS * RS_ROUNDS;

__global__ __launch_bounds__(RS_THREADS) void k_radix_hist(const uint32_t *__restrict__ keys, uint32_t n,
                                                           uint32_t shift, uint32_t *__restrict__ hist,
                                                           uint32_t nblk)
{
    __shared__ uint32_t h[256];
    const uint32_t tid = threadIdx.x;
    h[tid] = 0;
    __syncthreads();
    const uint32_t base = blockIdx.x * RS_TILE;
#pragma unroll
    for (int r = 0; r < RS_ROUNDS; ++r) {
        uint32_t i = base + r * RS_THREADS + tid;
        if (i < n) atomicAdd(&h[(keys[i] >> shift) & 255u], 1u);
    }
    __syncthreads();
    hist[tid * nblk + blockIdx.x] = h[tid];
}

// Per digit d (one block each): exclusive scan of hist[d][0 .. nblk) in place,
// digit total into tot[d].
__global__ __launch_bounds__(256) void k_radix_scan_digit(uint32_t *__restrict__ hist, uint32_t nblk,
                                                          uint32_t *__restrict__ tot)
{
    __shared__ uint32_t wsum[4];
    __shared__ uint32_t carry;
    const uint32_t tid = threadIdx.x, lane = tid & 63u, wv = tid >> 6;
    uint32_t *row = hist + (size_t)blockIdx.x * nblk;
    if (tid == 0) carry = 0;
    __syncthreads();
    for (uint32_t b0 = 0; b0 < nblk; b0 += 256) {
        const uint32_t i = b0 + tid;
        const uint32_t v = i < nblk ? row[i] : 0u;
        uint32_t inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d, 64);
            if (lane >= (uint32_t)d) inc += t;
        }
        if (lane == 63u) wsum[wv] = inc;
        __syncthreads();
        uint32_t before = carry;
        for (uint32_t w = 0; w < wv; ++w) before += wsum[w];
        if (i < nblk) row[i] = before + inc - v;
        __syncthreads();
        if (tid == 255u) carry = before + inc;
        __syncthreads();
    }
    if (tid == 0) tot[blockIdx.x] = carry;
}

// Stable scatter: elements are ranked in index order (round, wave, lane).
// Each block first turns the 256 digit totals into digit offsets (an
// exclusive scan, the same in every block).
__global__ __launch_bounds__(RS_THREADS) void k_radix_scatter(
    const uint32_t *__restrict__ kin, const uint32_t *__restrict__ vin, uint32_t *__restrict__ kout,
    uint32_t *__restrict__ vout, uint32_t n, uint32_t shift, const uint32_t *__restrict__ hist, uint32_t nblk,
    const uint32_t *__restrict__ tot)
{
    static_assert(RS_THREADS == 256, "one thread per digit");
    __shared__ uint32_t base[256];
    __shared__ uint32_t wcnt[RS_THREADS / 64][256];
    __shared__ uint32_t wsum[RS_THREADS / 64];
    const uint32_t tid = threadIdx.x;
    const uint32_t lane = tid & 63u, wv = tid >> 6;
    {
        const uint32_t v = tot[tid];
        uint32_t inc = v;
#pragma unroll
        for (int d = 1; d < 64; d <<= 1) {
            const uint32_t t = __shfl_up(inc, d, 64);
            if (lane >= (uint32_t)d) inc += t;
        }
        if (lane == 63u) wsum[wv] = inc;
        __syncthreads();
        uint32_t before = 0;
        for (uint32_t w = 0; w < wv; ++w) before += wsum[w];
        base[tid] = before + inc - v + hist[tid * nblk + blockIdx.x];
    }
    const uint64_t lt = (lane == 0) ? 0ull : (~0ull >> (64u - lane));
    const uint32_t tile = blockIdx.x * RS_TILE;
    for (int r = 0; r < RS_ROUNDS; ++r) {
        const uint32_t i = tile + r * RS_THREADS + tid;
        const bool valid = i < n;
        const uint32_t key = valid ? kin[i] : 0u;
        const uint32_t d = (key >> shift) & 255u;
        uint64_t peers = __ballot(valid);
#pragma unroll
        for (int bit = 0; bit < 8; ++bit) {
            const bool on = (d >> bit) & 1u;
            const uint64_t bb = __ballot(on);
            peers &= on ? bb : ~bb;
        }
        const uint32_t rank = __popcll(peers & lt);
        const uint32_t cnt = __popcll(peers);
#pragma unroll
        for (int w = 0; w < RS_THREADS / 64; ++w) wcnt[w][tid] = 0;
        __syncthreads();
        if (valid && rank == 0) wcnt[wv][d] = cnt;
        __syncthreads();
        {
            uint32_t run = base[tid];
#pragma unroll
            for (int w = 0; w < RS_THREADS / 64; ++w) {
                uint32_t c = wcnt[w][tid];
                wcnt[w][tid] = run;
                run += c;
            }
            base[tid] = run;
        }
        __syncthreads();
        if (valid) {
            const uint32_t pos = wcnt[wv][d] + rank;
            kout[pos] = key;
            vout[pos] = vin ? vin[i] : i;
        }
        __syncthreads();
    }
}

void launch_radix_sort(hipStream_t s, uint32_t n, int key_bits, Sort &st, uint32_t **sorted_keys,
                       uint32_t **sorted_vals)
{
    // keys start in keys_a with implicit values 0..n-1
    uint32_t *kin = st.keys_a, *kout = st.keys_b;
    uint32_t *vin = nullptr, *vout = st.vals_b;
    const uint32_t nblk = (n + RS_TILE - 1) / RS_TILE;
    int passes = (key_bits + 7) / 8;
    if (passes < 1) passes = 1;   // always produce the value permutation
    for (int p = 0; p < passes; ++p) {
        const uint32_t shift = 8u * (uint32_t)p;
        hipLaunchKernelGGL(k_radix_hist, dim3(nblk), dim3(RS_THREADS), 0, s, kin, n, shift, st.hist, nblk);
        hipLaunchKernelGGL(k_radix_scan_digit, dim3(256), dim3(256), 0, s, st.hist, nblk, st.dbase);
        hipLaunchKernelGGL(k_radix_scatter, dim3(nblk), dim3(RS_THREADS), 0, s, kin, vin, kout, vout, n,
                           shift, st.hist, nblk, st.dbase);
        // next pass reads what this one wrote
        uint32_t *nk = (kout == st.keys_b) ? st.keys_a : st.keys_b;
        uint32_t *nv = (vout == st.vals_b) ? st.vals_a : st.vals_b;
        kin = kout;
        vin = vout;
        kout = nk;
        vout = nv;
    }
    *sorted_keys = kin;
    *sorted_vals = vin;
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

// ---------------------------------------------------------------- reorder + cell table

template <typename T>
// Static boundary particles get density and force 0 in their new slot here:
// the neighbour passes never write them (a slot's previous particle may have).
__global__ __launch_bounds__(256) void k_reorder(uint32_t n, const uint32_t *__restrict__ perm,
                                                 const uint32_t *__restrict__ keys, State<T> in, State<T> out,
                                                 uint32_t *__restrict__ inv_perm, uint32_t *__restrict__ cstart,
                                                 uint32_t *__restrict__ cend, V2<T> *__restrict__ dens,
                                                 V4<T> *__restrict__ force)
{
    uint32_t p = blockIdx.x * 256u + threadIdx.x;
    if (p >= n) return;
    const uint32_t j = perm[p];
    out.pos[p] = in.pos[j];
    out.vel[p] = in.vel[j];
    const uint32_t id = in.id[j];
    out.id[p] = id;
    const uint32_t aux = in.aux[j];
    out.aux[p] = aux;
    if (aux_type(aux) == TY_BOUNDARY && !aux_kin(aux)) {
        dens[p] = V2<T>{(T)0, (T)0};
        force[p] = V4<T>{(T)0, (T)0, (T)0, (T)0};
    }
    inv_perm[id] = p;
    const uint32_t k = keys[p];
    if (p == 0 || keys[p - 1] != k) cstart[k] = p;
    if (p == n - 1 || keys[p + 1] != k) cend[k] = p + 1;
}

template <typename T>
void launch_reorder(hipStream_t s, uint32_t n, const uint32_t *perm, const uint32_t *keys, State<T> in,
                    State<T> out, uint32_t *inv_perm, uint32_t *cstart, uint32_t *cend, V2<T> *dens, V4<T> *force)
{
    if (!n) return;
    hipLaunchKernelGGL(k_reorder<T>, dim3((n + 255) / 256), dim3(256), 0, s, n, perm, keys, in, out, inv_perm,
                       cstart, cend, dens, force);
}
template void launch_reorder<float>(hipStream_t, uint32_t, const uint32_t *, const uint32_t *, State<float>,
                                    State<float>, uint32_t *, uint32_t *, uint32_t *, V2<float> *, V4<float> *);
template void launch_reorder<double>(hipStream_t, uint32_t, const uint32_t *, const uint32_t *, State<double>,
                                     State<double>, uint32_t *, uint32_t *, uint32_t *, V2<double> *, V4<double> *);

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
