// Split step: one bond kernel per lattice axis writes every bond's result
// (force on voxel 2, moments on both ends) to a scratch buffer, then one
// gather kernel sums each voxel's at most six bonds in a fixed order and
// integrates.  Simple and atomic-free; the fused kernel computes the same
// per-bond and per-voxel arithmetic without the scratch round trip.
#include "vx_adjoint.hpp"
#include "vx_launch.hpp"

namespace vx {

template <typename T, int AX>
__global__ void __launch_bounds__(256) k_bonds(StepArgs<T> a) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const uint8_t ma = a.mat[c];
    if (ma == 0) return;
    const long long nxy = (long long)a.nx * a.ny;
    long long cn;
    if (AX == 0) {
        if ((int)(c % a.nx) + 1 >= a.nx) return;
        cn = c + 1;
    } else if (AX == 1) {
        if ((int)((c / a.nx) % a.ny) + 1 >= a.ny) return;
        cn = c + a.nx;
    } else {
        if ((int)(c / nxy) + 1 >= a.nz) return;
        cn = c + nxy;
    }
    const uint8_t mb = a.mat[cn];
    if (mb == 0) return;
    const MatConst<T> A = mat_at(a, c, ma), B = mat_at(a, cn, mb);
    const T ea = voxel_strain(a, (unsigned)c, a.flags[c], A.cte);
    const T eb = voxel_strain(a, (unsigned)cn, a.flags[cn], B.cte);
    const VoxKin<T> ka = load_kin(a.s_in, a.stride, (unsigned)c, A, ea);
    const VoxKin<T> kb = load_kin(a.s_in, a.stride, (unsigned)cn, B, eb);
    const Rot<T> R = rot_of(ka.qw, ka.qx, ka.qy, ka.qz);
    const LatK<T> C = lat_consts(a.l);
    const BondK<T> K = a.E_cell ? bond_k_from_E(a.E_cell[c], a.E_cell[cn], A.gfac, B.gfac, A.m < B.m ? A.m : B.m,
                                                a.zeta_bond, C)
                                : bond_k(a.pairs[ma * a.n_mat + mb]);
    const BondOut<T> o = bond_eval<T, AX>(ka, R, kb, K, C);
    T *b = a.bonds + (long long)AX * 9 * a.stride;
    const long long st = a.stride;
    b[0 * st + c] = o.f2x; b[1 * st + c] = o.f2y; b[2 * st + c] = o.f2z;
    b[3 * st + c] = o.m1x; b[4 * st + c] = o.m1y; b[5 * st + c] = o.m1z;
    b[6 * st + c] = o.m2x; b[7 * st + c] = o.m2y; b[8 * st + c] = o.m2z;
}

template <typename T>
__global__ void __launch_bounds__(256) k_gather(StepArgs<T> a) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const long long c = (long long)blockIdx.x * blockDim.x + threadIdx.x;
    T vmax = T(0);
    if (c < n) {
        const uint8_t m = a.mat[c];
        if (m != 0) {
            const long long nxy = (long long)a.nx * a.ny;
            const int ix = (int)(c % a.nx), iy = (int)((c / a.nx) % a.ny), iz = (int)(c / nxy);
            const long long st = a.stride;
            T Fx = T(0), Fy = T(0), Fz = T(0), Mx = T(0), My = T(0), Mz = T(0);
            const int idx[3] = {ix, iy, iz};
            const int dim[3] = {a.nx, a.ny, a.nz};
            const long long step[3] = {1, a.nx, nxy};
#pragma unroll
            for (int ax = 0; ax < 3; ++ax) {
                const T *b = a.bonds + (long long)ax * 9 * st;
                if (idx[ax] > 0 && a.mat[c - step[ax]] != 0) {  // this voxel is voxel 2
                    const long long cb = c - step[ax];
                    Fx += b[0 * st + cb]; Fy += b[1 * st + cb]; Fz += b[2 * st + cb];
                    Mx += b[6 * st + cb]; My += b[7 * st + cb]; Mz += b[8 * st + cb];
                }
                if (idx[ax] + 1 < dim[ax] && a.mat[c + step[ax]] != 0) {  // voxel 1
                    Fx -= b[0 * st + c]; Fy -= b[1 * st + c]; Fz -= b[2 * st + c];
                    Mx += b[3 * st + c]; My += b[4 * st + c]; Mz += b[5 * st + c];
                }
            }
            const MatConst<T> mc = mat_at(a, c, m);
            const uint8_t fl = a.flags[c];
            const T eps = voxel_strain(a, (unsigned)c, fl, mc.cte);
            if (a.fm_out) {
                a.fm_out[0 * st + c] = Fx; a.fm_out[1 * st + c] = Fy; a.fm_out[2 * st + c] = Fz;
                a.fm_out[3 * st + c] = Mx; a.fm_out[4 * st + c] = My; a.fm_out[5 * st + c] = Mz;
            }
            const VoxRaw<T> r = load_raw(a.s_in, st, (unsigned)c);
            voxel_update(a, (unsigned)c, fl, mc, eps, r, Fx, Fy, Fz, Mx, My, Mz, &vmax);
        }
    }
    if (a.track_vmax) wave_vmax(a.vmax_bits, vmax);
}

template <typename T>
hipError_t launch_split_step(const StepArgs<T> &a, hipStream_t s) {
    const long long n = (long long)a.nx * a.ny * a.nz;
    const unsigned blocks = (unsigned)((n + 255) / 256);
    k_bonds<T, 0><<<blocks, 256, 0, s>>>(a);
    k_bonds<T, 1><<<blocks, 256, 0, s>>>(a);
    k_bonds<T, 2><<<blocks, 256, 0, s>>>(a);
    k_gather<T><<<blocks, 256, 0, s>>>(a);
    return hipGetLastError();
}

template hipError_t launch_split_step<float>(const StepArgs<float> &, hipStream_t);
template hipError_t launch_split_step<double>(const StepArgs<double> &, hipStream_t);

}  // namespace vx
