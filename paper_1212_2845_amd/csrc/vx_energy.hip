// Whole-lattice energies and momenta of the current state: one thread per
// cell accumulates its kinetic, gravitational and floor energies, its
// momentum and angular momentum about the world origin, and the elastic
// energy of the (at most three) bonds it is voxel 1 of; a fixed-order tree
// in LDS reduces each workgroup to one row of FP64 partials, which the host
// sums in workgroup order.  Deterministic, no atomics.
#include "vx_adjoint.hpp"
#include "vx_launch.hpp"

namespace vx {

namespace {

constexpr int kEnergyThreads = 256;

// Elastic energy of one bond, 1/2 u2^T K22 u2 with u2 = (X2, Y2, Z2, theta)
// of voxel 2 in voxel 1's bond frame and K22 the lower-right block of Eq. 7
// (the same local coordinates as bond_core).
template <typename T, int AX>
__device__ double bond_energy(const VoxKin<T> &A, const Rot<T> &R, const VoxKin<T> &B, const BondK<T> &K,
                              const LatK<T> &C) {
    constexpr int A0 = AX, A1 = (AX + 1) % 3, A2 = (AX + 2) % 3;
    const T du[3] = {B.ux - A.ux, B.uy - A.uy, B.uz - A.uz};
    T th[3];
    rel_rotvec(A, B, th);
    const V3<T> ex = R.c[A0], ey = R.c[A1], ez = R.c[A2];
    const double X2 = ex.x * du[0] + ex.y * du[1] + ex.z * du[2] + C.l * (R.dm1[A0] - T(0.5) * (A.eps + B.eps));
    const double Y2 = ey.x * du[0] + ey.y * du[1] + ey.z * du[2] + C.l * comp<AX>(ey);
    const double Z2 = ez.x * du[0] + ez.y * du[1] + ez.z * du[2] + C.l * comp<AX>(ez);
    const double tx = th[A0], ty = th[A1], tz = th[A2];
    const double a1 = K.a1, a2 = K.a2, l = C.l;
    const double b2 = a1 * 0.5 * l, b3 = a1 * l * l / 6.0;
    return 0.5 * (a1 * X2 * X2 + a1 * Y2 * Y2 + a1 * Z2 * Z2 + a2 * tx * tx + 2.0 * b3 * ty * ty +
                  2.0 * b3 * tz * tz) + b2 * Z2 * ty - b2 * Y2 * tz;
}

template <typename T>
__device__ __forceinline__ BondK<T> bond_at(const StepArgs<T> &a, long long c, long long cn, uint8_t ma, uint8_t mb,
                                            const MatConst<T> &A, const MatConst<T> &B, const LatK<T> &C) {
    return a.E_cell ? bond_k_from_E(a.E_cell[c], a.E_cell[cn], A.gfac, B.gfac, A.m < B.m ? A.m : B.m, a.zeta_bond, C)
                    : bond_k(a.pairs[ma * a.n_mat + mb]);
}

template <typename T>
__global__ void __launch_bounds__(kEnergyThreads) k_energy(StepArgs<T> a, double *partials) {
    __shared__ double red[kEnergyWords][kEnergyThreads];
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    double acc[kEnergyWords];
#pragma unroll
    for (int i = 0; i < kEnergyWords; ++i) acc[i] = 0.0;
    if (c < n && a.mat[c] != 0) {
        const uint8_t m = a.mat[c];
        const long long st = a.stride, nxy = (long long)a.nx * a.ny;
        const int idx[3] = {(int)(c % a.nx), (int)((c / a.nx) % a.ny), (int)(c / nxy)};
        const int dim[3] = {a.nx, a.ny, a.nz};
        const long long stp[3] = {1, a.nx, nxy};
        const MatConst<T> mc = mat_at(a, c, m);
        const uint8_t fl = a.flags[c];
        const T eps = voxel_strain(a, (unsigned)c, fl, mc.cte);
        const VoxRaw<T> r = load_raw(a.s_in, st, (unsigned)c);
        const double P[3] = {r.px, r.py, r.pz}, Lw[3] = {r.lx, r.ly, r.lz};
        const double mass = mc.m, I = mc.I, l = a.l;
        acc[0] = 0.5 * (P[0] * P[0] + P[1] * P[1] + P[2] * P[2]) / mass +
                 0.5 * (Lw[0] * Lw[0] + Lw[1] * Lw[1] + Lw[2] * Lw[2]) / I;
        const double pos[3] = {a.origin[0] + (idx[0] + 0.5) * l + (double)r.ux,
                               a.origin[1] + (idx[1] + 0.5) * l + (double)r.uy,
                               a.origin[2] + (idx[2] + 0.5) * l + (double)r.uz};
        acc[2] = mass * (double)a.gravity * pos[2];
        if (a.floor_on) {
            const double pen = 0.5 * l * (double)eps - (double)r.uz - ((double)a.origin_z + idx[2] * l);
            if (pen > 0.0) acc[3] = 0.5 * (double)mc.kv * pen * pen;
        }
        acc[4] = P[0]; acc[5] = P[1]; acc[6] = P[2];
        acc[7] = pos[1] * P[2] - pos[2] * P[1] + Lw[0];
        acc[8] = pos[2] * P[0] - pos[0] * P[2] + Lw[1];
        acc[9] = pos[0] * P[1] - pos[1] * P[0] + Lw[2];
        // bonds this voxel is voxel 1 of
        const VoxKin<T> ka = kin_of(r, mc, eps);
        const Rot<T> R = rot_of(ka.qw, ka.qx, ka.qy, ka.qz);
        const LatK<T> C = lat_consts(a.l);
        double ue = 0.0;
#pragma unroll
        for (int ax = 0; ax < 3; ++ax) {
            if (idx[ax] + 1 >= dim[ax]) continue;
            const long long cn = c + stp[ax];
            const uint8_t mb = a.mat[cn];
            if (!mb) continue;
            const MatConst<T> B = mat_at(a, cn, mb);
            const T eb = voxel_strain(a, (unsigned)cn, a.flags[cn], B.cte);
            const VoxKin<T> kb = load_kin(a.s_in, st, (unsigned)cn, B, eb);
            const BondK<T> K = bond_at(a, c, cn, m, mb, mc, B, C);
            if (ax == 0) ue += bond_energy<T, 0>(ka, R, kb, K, C);
            else if (ax == 1) ue += bond_energy<T, 1>(ka, R, kb, K, C);
            else ue += bond_energy<T, 2>(ka, R, kb, K, C);
        }
        acc[1] = ue;
    }
#pragma unroll
    for (int i = 0; i < kEnergyWords; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = kEnergyThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int i = 0; i < kEnergyWords; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kEnergyWords) partials[(long long)blockIdx.x * kEnergyWords + threadIdx.x] = red[threadIdx.x][0];
}

// Sum of the per-workgroup partials of k_energy into out[0..kEnergyWords),
// on the device, in a fixed order: thread t adds rows t, t + 256, ... in
// turn, then a fixed tree over the threads.
__global__ void __launch_bounds__(kEnergyThreads) k_energy_sum(const double *partials, int nb, double *out) {
    __shared__ double red[kEnergyWords][kEnergyThreads];
    double acc[kEnergyWords];
#pragma unroll
    for (int i = 0; i < kEnergyWords; ++i) acc[i] = 0.0;
    for (int b = threadIdx.x; b < nb; b += kEnergyThreads)
#pragma unroll
        for (int i = 0; i < kEnergyWords; ++i) acc[i] += partials[(long long)b * kEnergyWords + i];
#pragma unroll
    for (int i = 0; i < kEnergyWords; ++i) red[i][threadIdx.x] = acc[i];
    __syncthreads();
    for (int s = kEnergyThreads / 2; s > 0; s >>= 1) {
        if ((int)threadIdx.x < s)
#pragma unroll
            for (int i = 0; i < kEnergyWords; ++i) red[i][threadIdx.x] += red[i][threadIdx.x + s];
        __syncthreads();
    }
    if (threadIdx.x < kEnergyWords) out[threadIdx.x] = red[threadIdx.x][0];
}

// One state word of listed cells into a device array: the recording step of
// a long run (e.g. a probe voxel's displacement every few steps for a modal
// spectrum) without a host synchronisation.  An index outside the lattice
// reads as NaN.
template <typename T>
__global__ void __launch_bounds__(256) k_probe(const T *__restrict__ state, long long stride, long long ncell,
                                               const int32_t *__restrict__ cells, int n, int word,
                                               T *__restrict__ out) {
    const int i = blockIdx.x * 256 + threadIdx.x;
    if (i >= n) return;
    const int32_t c = cells[i];
    out[i] = (c >= 0 && (long long)c < ncell) ? state[(long long)word * stride + c] : T(__builtin_nan(""));
}

}  // namespace

template <typename T>
hipError_t launch_probe(const T *state, long long stride, long long ncell, const int32_t *cells, int n, int word,
                        T *out, hipStream_t s) {
    if (n <= 0) return hipSuccess;
    k_probe<T><<<(unsigned)((n + 255) / 256), 256, 0, s>>>(state, stride, ncell, cells, n, word, out);
    return hipGetLastError();
}

template hipError_t launch_probe<float>(const float *, long long, long long, const int32_t *, int, int, float *,
                                        hipStream_t);
template hipError_t launch_probe<double>(const double *, long long, long long, const int32_t *, int, int,
                                         double *, hipStream_t);

int energy_blocks(long long ncell) { return (int)((ncell + kEnergyThreads - 1) / kEnergyThreads); }

template <typename T>
hipError_t launch_energy(const StepArgs<T> &a, double *partials, hipStream_t s) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    k_energy<T><<<energy_blocks(n), kEnergyThreads, 0, s>>>(a, partials);
    return hipGetLastError();
}

hipError_t launch_energy_sum(const double *partials, long long ncell, double *out, hipStream_t s) {
    k_energy_sum<<<1, kEnergyThreads, 0, s>>>(partials, energy_blocks(ncell), out);
    return hipGetLastError();
}

template hipError_t launch_energy<float>(const StepArgs<float> &, double *, hipStream_t);
template hipError_t launch_energy<double>(const StepArgs<double> &, double *, hipStream_t);

}  // namespace vx
