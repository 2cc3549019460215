// Rigid bodies and the integrator of one SPH step (arXiv 2511.15908):
//  - kinematic (grabbed) bodies: the pose comes from the haptic device
//    (Sec. 3.3, Fig. 1); their particles keep constant offsets from it
//    (Sec. 3.2) and are placed by the key launch (place_body_particle);
//  - body wrench: the particles' point forces summed into the parent's force
//    and torque (Sec. 3.2, Alg. 2: the rigid-force step), reduced in
//    binary64 by one block per body in a fixed order (deterministic), pushed
//    into the rolling-average ring of Sec. 3.3; it runs in the integration
//    launch;
//  - semi-implicit Euler (Eq. euler) for fluid and soft particles.
// (The soft bodies' spring forces run in the density launch, k_sums.hip.)
#include "sph_internal.h"

namespace sphk {


// ------------------------------------------------------------------ wrench

__device__ __forceinline__ double wave_sum(double v)
{
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) v += __shfl_xor(v, m, 64);
    return v;
}

// The wrench of kinematic object o (Sec. 3.2: the rigid particles' point
// forces summed into the parent body), one 256-thread block per object, in
// the integration launch: each thread sums the object's body particles t,
// t + 256, ... in order, the block adds its four wavefront sums in a fixed
// order, and thread 0 pushes the sample into the ring, logs the step and
// advances the pose (wrench_apply).  No block depends on another, so no
// cross-block fence is needed and the result does not depend on the order
// in which blocks run.
// The step's sample of object o: ring, log, free-body dynamics, next pose.
__device__ __forceinline__ void wrench_apply(const BodyArgs &b, uint32_t o, const double v[6])
{
#pragma clang fp contract(off)
    {
        const uint32_t cnt = b.ring_count[o];
        double *slot = b.ring + ((size_t)o * b.K + (cnt % b.K)) * 6u;
        for (int c = 0; c < 6; ++c) slot[c] = v[c];
        b.ring_count[o] = cnt + 1u;
        double *pz = b.poses + 16u * o;
        const double dt = b.dt;
        if (b.log_cap) {
            // the step's record: the pose and velocities the forces saw, the wrench
            const uint32_t row = b.log_count[o];
            double *r = b.log + ((size_t)(row % b.log_cap) * b.nk + o) * 20u;
            for (int a = 0; a < 13; ++a) r[a] = pz[a];
            for (int c = 0; c < 6; ++c) r[13 + c] = v[c];
            r[19] = (double)row;
            b.log_count[o] = row + 1u;
        }
        if (b.props && b.props[24u * o + kPropFree] != 0.0) {
            // free body: v += dt (F/m + g); w += dt I_w^-1 (T - w x I_w w),
            // I_w = R I R^T and I_w^-1 = R I^-1 R^T (Euler's equations)
            const double *pr = b.props + 24u * o;
            double R[9];
            quat_R(pz + 3, R);
            double Iw[9], Iwi[9];
            for (int r = 0; r < 3; ++r)
                for (int c2 = 0; c2 < 3; ++c2) {
                    double a1 = 0.0, a2 = 0.0;
                    for (int k = 0; k < 3; ++k)
                        for (int l = 0; l < 3; ++l) {
                            a1 += R[3 * r + k] * pr[1 + 3 * k + l] * R[3 * c2 + l];
                            a2 += R[3 * r + k] * pr[10 + 3 * k + l] * R[3 * c2 + l];
                        }
                    Iw[3 * r + c2] = a1;
                    Iwi[3 * r + c2] = a2;
                }
            const double w0 = pz[10], w1 = pz[11], w2 = pz[12];
            const double L0 = Iw[0] * w0 + Iw[1] * w1 + Iw[2] * w2;
            const double L1 = Iw[3] * w0 + Iw[4] * w1 + Iw[5] * w2;
            const double L2 = Iw[6] * w0 + Iw[7] * w1 + Iw[8] * w2;
            const double r0 = v[3] - (w1 * L2 - w2 * L1);
            const double r1 = v[4] - (w2 * L0 - w0 * L2);
            const double r2 = v[5] - (w0 * L1 - w1 * L0);
            for (int a = 0; a < 3; ++a) {
                pz[7 + a] = pz[7 + a] + dt * (v[a] / pr[0] + b.g[a]);
                pz[10 + a] = pz[10 + a] + dt * (Iwi[3 * a] * r0 + Iwi[3 * a + 1] * r1 + Iwi[3 * a + 2] * r2);
            }
        }
        if (b.track && b.track_pos[2u * o] < b.track_pos[2u * o + 1u]) {
            // next pose of the body's track
            const uint32_t k = b.track_pos[2u * o];
            const double *tp = b.track + ((size_t)o * b.track_cap + k) * 16u;
            for (int a = 0; a < 13; ++a) pz[a] = tp[a];
            b.track_pos[2u * o] = k + 1u;
            return;
        }
        // pose advance: c += v dt, q <- normalise(q + dt/2 (0, w) q)
        for (int a = 0; a < 3; ++a) pz[a] = pz[a] + pz[7 + a] * dt;
        const double qw = pz[3], qx = pz[4], qy = pz[5], qz = pz[6];
        const double wx = pz[10], wy = pz[11], wz = pz[12];
        const double d0 = -wx * qx - wy * qy - wz * qz;
        const double d1 = wx * qw + wy * qz - wz * qy;
        const double d2 = wy * qw + wz * qx - wx * qz;
        const double d3 = wz * qw + wx * qy - wy * qx;
        const double n0 = qw + 0.5 * dt * d0, n1 = qx + 0.5 * dt * d1;
        const double n2 = qy + 0.5 * dt * d2, n3 = qz + 0.5 * dt * d3;
        const double s = sqrt(n0 * n0 + n1 * n1 + n2 * n2 + n3 * n3);
        pz[3] = n0 / s;
        pz[4] = n1 / s;
        pz[5] = n2 / s;
        pz[6] = n3 / s;
    }
}


struct PoseArg {
    double v[13];
};

__global__ void k_set_pose(double *__restrict__ slot, PoseArg a)
{
    const uint32_t t = threadIdx.x;
    if (t < 13) slot[t] = a.v[t];
}

void launch_set_pose(hipStream_t s, double *pose_slot, const double c[3], const double q[4], const double v[3],
                     const double w[3])
{
    PoseArg a;
    for (int k = 0; k < 3; ++k) a.v[k] = c[k];
    for (int k = 0; k < 4; ++k) a.v[3 + k] = q[k];
    for (int k = 0; k < 3; ++k) a.v[7 + k] = v[k];
    for (int k = 0; k < 3; ++k) a.v[10 + k] = w[k];
    hipLaunchKernelGGL(k_set_pose, dim3(1), dim3(64), 0, s, pose_slot, a);
}

__global__ void k_reset_ring(uint32_t *__restrict__ cnt)
{
    if (threadIdx.x == 0) cnt[0] = 0u;
}

void launch_reset_ring(hipStream_t s, uint32_t *ring_count_slot)
{
    hipLaunchKernelGGL(k_reset_ring, dim3(1), dim3(64), 0, s, ring_count_slot);
}

__global__ void k_set_double(double *__restrict__ slot, double v)
{
    if (threadIdx.x == 0) slot[0] = v;
}

void launch_set_double(hipStream_t s, double *slot, double v)
{
    hipLaunchKernelGGL(k_set_double, dim3(1), dim3(64), 0, s, slot, v);
}

__global__ void k_set_u32x2(uint32_t *__restrict__ slot, uint32_t a, uint32_t b)
{
    if (threadIdx.x == 0) {
        slot[0] = a;
        slot[1] = b;
    }
}

void launch_set_u32x2(hipStream_t s, uint32_t *slot, uint32_t a, uint32_t b)
{
    hipLaunchKernelGGL(k_set_u32x2, dim3(1), dim3(64), 0, s, slot, a, b);
}

// ------------------------------------------------------------------ density probes

// rho(p) = sum over fluid/soft j with predicate(p, x_j) of m_j W(|p - x_j|):
// the density field of Sec. 3.4 at arbitrary points, through the cell table.
// One wavefront per probe: the lanes stride over the particles of each of the
// 27 cells (coalesced loads), FP64 partial sums, fixed shuffle-tree reduction.
template <typename T>
__global__ __launch_bounds__(64) void k_probe(ProbeArgs a, State<T> st, Batch<T> b,
                                              const uint32_t *__restrict__ cstart,
                                              const uint32_t *__restrict__ cend)
{
#pragma clang fp contract(off)
    const uint32_t i = blockIdx.x, lane = threadIdx.x;
    if (i >= a.n) return;
    const uint32_t si = a.scene[i];    // the probe's scene: its grid, constants and cells
    const Grid g = b.sc[si].g;
    const Phys<T> ph = b.sc[si].ph;
    double p[3] = {a.pts[3 * i], a.pts[3 * i + 1], a.pts[3 * i + 2]};
    const int32_t f = a.frame[i];
    if (f >= 0) {
        const double *pose = a.poses + 16 * f;
        double R[9];
        quat_R(pose + 3, R);
        double w[3];
        for (int k = 0; k < 3; ++k) w[k] = R[3 * k] * p[0] + R[3 * k + 1] * p[1] + R[3 * k + 2] * p[2];
        for (int k = 0; k < 3; ++k) p[k] = pose[k] + w[k];
    }
    const V4<T> me{(T)p[0], (T)p[1], (T)p[2], (T)0};
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
        for (uint32_t j = cstart[key] + lane; j < e; j += 64u) {
            const V4<T> c = st.pos[j];
            if (c.w < (T)0 || aux_type(st.aux[j]) == TY_BOUNDARY) continue;
            if (!within_support<T>(me, c, R2)) continue;
            acc += (double)c.w * kernel_w64<T>(c, me, ph);
        }
    }
#pragma unroll
    for (int m = 32; m >= 1; m >>= 1) acc += __shfl_xor(acc, m, 64);
    if (lane == 0) {
        a.out[i] = acc;
        // the body log's wrench pass of this step runs later and advances the row
        if (a.log) a.log[(size_t)(*a.log_row % a.log_cap) * a.stride + i] = acc;
    }
}

template <typename T>
void launch_probe(hipStream_t s, const ProbeArgs &a, State<T> st, const Batch<T> &b, const uint32_t *cstart,
                  const uint32_t *cend)
{
    if (!a.n) return;
    hipLaunchKernelGGL(k_probe<T>, dim3(a.n), dim3(64), 0, s, a, st, b, cstart, cend);
}
template void launch_probe<float>(hipStream_t, const ProbeArgs &, State<float>, const Batch<float> &,
                                  const uint32_t *, const uint32_t *);
template void launch_probe<double>(hipStream_t, const ProbeArgs &, State<double>, const Batch<double> &,
                                   const uint32_t *, const uint32_t *);

// ------------------------------------------------------------------ integrate

__device__ __forceinline__ void wrench_obj(const BodyArgs &b, uint32_t o)
{
    __shared__ double red[4][6];
    const uint32_t t = threadIdx.x, lane = t & 63u, wv = t >> 6;
    double R[9];
    quat_R(b.poses + 16u * o + 3, R);
    double v[6] = {0, 0, 0, 0, 0, 0};
    // unrolled: the loads of four particles are in flight together
#pragma unroll 4
    for (uint32_t s = b.obj_slot0[o] + t; s < b.obj_slot0[o + 1]; s += 256u) {
        const double r0 = b.r_loc[3 * s], r1 = b.r_loc[3 * s + 1], r2 = b.r_loc[3 * s + 2];
        double rw[3];
        for (int a = 0; a < 3; ++a) rw[a] = R[3 * a] * r0 + R[3 * a + 1] * r1 + R[3 * a + 2] * r2;
        const double fx = b.fbody[3 * s], fy = b.fbody[3 * s + 1], fz = b.fbody[3 * s + 2];
        v[0] += fx;
        v[1] += fy;
        v[2] += fz;
        v[3] += rw[1] * fz - rw[2] * fy;
        v[4] += rw[2] * fx - rw[0] * fz;
        v[5] += rw[0] * fy - rw[1] * fx;
    }
#pragma unroll
    for (int k = 0; k < 6; ++k) v[k] = wave_sum(v[k]);
    if (lane == 0)
        for (int k = 0; k < 6; ++k) red[wv][k] = v[k];
    __syncthreads();
    if (t != 0) return;
    double w[6];
    for (int k = 0; k < 6; ++k) w[k] = ((red[0][k] + red[1][k]) + red[2][k]) + red[3][k];
    wrench_apply(b, o, w);
}


// Blocks [0, nw) reduce the wrench of one kinematic object each (above, from
// the same step's forces), the blocks after them integrate the particles.
template <typename T>
__global__ __launch_bounds__(256) void k_integrate(uint32_t n, uint32_t nw, State<T> st,
                                                   const V4<T> *__restrict__ force, Phys<T> ph,
                                                   uint32_t *__restrict__ err, BodyArgs b)
{
    if (blockIdx.x < nw) {
        wrench_obj(b, blockIdx.x);
        return;
    }
    const uint32_t p = (blockIdx.x - nw) * 256u + threadIdx.x;
    if (p >= n) return;
    if (aux_type(st.aux[p]) == TY_BOUNDARY) return;
    V4<T> x = st.pos[p];
    V4<T> v = st.vel[p];
    const V4<T> f = force[p];
    const T m = x.w;
    v.x = v.x + (f.x / m) * ph.dt;
    v.y = v.y + (f.y / m) * ph.dt;
    v.z = v.z + (f.z / m) * ph.dt;
    x.x = x.x + v.x * ph.dt;
    x.y = x.y + v.y * ph.dt;
    x.z = x.z + v.z * ph.dt;
    st.pos[p] = x;
    st.vel[p] = v;
    const T v2 = v.x * v.x + v.y * v.y + v.z * v.z;
    const bool bad = !(v2 == v2) || !isfinite(v2) || !isfinite(x.x) || !isfinite(x.y) || !isfinite(x.z) ||
                     (ph.vmax2 > (T)0 && v2 > ph.vmax2);
    if (bad) atomicOr(err, ERR_UNSTABLE);
}

template <typename T>
void launch_integrate(hipStream_t s, uint32_t n, State<T> st, const V4<T> *force, const Phys<T> &ph, uint32_t *err,
                      const BodyArgs &b)
{
    if (!n) return;
    const uint32_t nint = (n + 255) / 256;
    hipLaunchKernelGGL(k_integrate<T>, dim3(b.nk + nint), dim3(256), 0, s, n, b.nk, st, force, ph, err, b);
}
template void launch_integrate<float>(hipStream_t, uint32_t, State<float>, const V4<float> *, const Phys<float> &,
                                      uint32_t *, const BodyArgs &);
template void launch_integrate<double>(hipStream_t, uint32_t, State<double>, const V4<double> *,
                                       const Phys<double> &, uint32_t *, const BodyArgs &);

}  // namespace sphk
