// Self-collision (section "Self collision detection and handling"):
// surface voxels only, a candidate list of pairs inside the collision
// horizon (centre distance < 2 l) excluding lattice neighbours within
// Manhattan distance 3, rebuilt only when the accumulated maximum motion
// could let an unlisted pair touch, and a per-step contact force from each
// voxel's own sorted list (every pair is evaluated from both sides, so no
// atomics touch the forces).
//
// Candidate search is a uniform grid of cell size = horizon, hashed into a
// power-of-two table and bucketed by a counting sort (count, scan,
// scatter).  Bucket order is not deterministic; each voxel's list is kept
// sorted by partner cell, so the lists themselves are.
#include <algorithm>

#include "vx_device.hpp"
#include "vx_launch.hpp"

namespace vx {

namespace {

constexpr int kScanBlock = 1024;   // entries per scan block (256 threads x 4)

__device__ __forceinline__ int cell_hash(int cx, int cy, int cz, int mask) {
    const unsigned h = ((unsigned)cx * 73856093u) ^ ((unsigned)cy * 19349663u) ^ ((unsigned)cz * 83492791u);
    return (int)(h & (unsigned)mask);
}

template <typename T>
__device__ __forceinline__ void voxel_pos(const StepArgs<T> &a, int c, int &ix, int &iy, int &iz, T &x, T &y,
                                          T &z, const T *origin) {
    ix = c % a.nx;
    iy = (c / a.nx) % a.ny;
    iz = c / (a.nx * a.ny);
    x = origin[0] + (T(ix) + T(0.5)) * a.l + a.s_in[W_UX * a.stride + c];
    y = origin[1] + (T(iy) + T(0.5)) * a.l + a.s_in[W_UY * a.stride + c];
    z = origin[2] + (T(iz) + T(0.5)) * a.l + a.s_in[W_UZ * a.stride + c];
}

struct Origin3 { double v[3]; };

template <typename T>
__device__ __forceinline__ void grid_cell(T x, T y, T z, double H, int &cx, int &cy, int &cz) {
    cx = (int)floor((double)x / H);
    cy = (int)floor((double)y / H);
    cz = (int)floor((double)z / H);
}

// Three integers of at most 21 bits each (offset by 2^20, so grid cells a
// little below the origin pack too) in one 64-bit word.  Two neighbouring
// grid cells never share a packed value.
__device__ __forceinline__ long long pack3(int x, int y, int z) {
    const unsigned long long m = 0x1FFFFFull, b = 1ull << 20;
    return (long long)((((unsigned long long)(x + (int)b)) & m) | ((((unsigned long long)(y + (int)b)) & m) << 21) |
                       ((((unsigned long long)(z + (int)b)) & m) << 42));
}

__device__ __forceinline__ void unpack3(long long v, int &x, int &y, int &z) {
    const unsigned long long u = (unsigned long long)v, m = 0x1FFFFFull;
    const int b = 1 << 20;
    x = (int)(u & m) - b;
    y = (int)((u >> 21) & m) - b;
    z = (int)((u >> 42) & m) - b;
}

// Surface voxels per workgroup of the candidate search (27 threads each),
// and the largest grid of the rebuild kernels (they stride over their work).
constexpr int kCandVox = 9;
constexpr int kCandGrid = 512;
// bucket entries whose loads the candidate search issues together
constexpr int kGroup = 4;

template <typename T>
__global__ void __launch_bounds__(256) k_keys(StepArgs<T> a, CollideArgs c, Origin3 o) {
    if (*c.rebuild_flag == 0) return;
    const int first = blockIdx.x * blockDim.x + threadIdx.x;
    if (first == 0) *c.pair_count = 0ull;
    const T org[3] = {(T)o.v[0], (T)o.v[1], (T)o.v[2]};
    for (int i = first; i < c.n_surf; i += gridDim.x * blockDim.x) {
        int ix, iy, iz, cx, cy, cz;
        T x, y, z;
        voxel_pos(a, c.surf_cells[i], ix, iy, iz, x, y, z, org);
        grid_cell(x, y, z, c.horizon, cx, cy, cz);
        const int key = cell_hash(cx, cy, cz, c.table_size - 1);
        c.cell_keys[i] = key;
        c.cell_gc[i] = pack3(cx, cy, cz);
        c.cell_ijk[i] = pack3(ix, iy, iz);
        atomicAdd(&c.bucket_fill[key], 1);
    }
}

// Scan of bucket counts -> bucket_start (exclusive), in three phases.
__global__ void __launch_bounds__(256) k_scan_reduce(CollideArgs c) {
    if (*c.rebuild_flag == 0) return;
    __shared__ int red[256];
    const int base = blockIdx.x * kScanBlock;
    int s = 0;
    for (int k = 0; k < 4; ++k) {
        const int j = base + threadIdx.x * 4 + k;
        if (j < c.table_size) s += c.bucket_fill[j];
    }
    red[threadIdx.x] = s;
    __syncthreads();
    for (int off = 128; off > 0; off >>= 1) {
        if ((int)threadIdx.x < off) red[threadIdx.x] += red[threadIdx.x + off];
        __syncthreads();
    }
    if (threadIdx.x == 0) ((int *)c.scan_tmp)[blockIdx.x] = red[0];
}

__global__ void __launch_bounds__(1024) k_scan_blocks(CollideArgs c, int nblocks) {
    if (*c.rebuild_flag == 0) return;
    __shared__ int buf[1024];
    __shared__ int carry;
    int *bs = (int *)c.scan_tmp;
    if (threadIdx.x == 0) carry = 0;
    __syncthreads();
    for (int base = 0; base < nblocks; base += 1024) {
        const int j = base + threadIdx.x;
        const int v = j < nblocks ? bs[j] : 0;
        buf[threadIdx.x] = v;
        __syncthreads();
        // Hillis-Steele inclusive scan
        for (int off = 1; off < 1024; off <<= 1) {
            const int t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
            __syncthreads();
            buf[threadIdx.x] += t;
            __syncthreads();
        }
        if (j < nblocks) bs[j] = carry + buf[threadIdx.x] - v;   // exclusive
        __syncthreads();
        if (threadIdx.x == 1023) carry += buf[1023];
        __syncthreads();
    }
}

__global__ void __launch_bounds__(256) k_scan_apply(CollideArgs c) {
    if (*c.rebuild_flag == 0) return;
    __shared__ int buf[256];
    const int base = blockIdx.x * kScanBlock;
    int v[4], s = 0;
    for (int k = 0; k < 4; ++k) {
        const int j = base + threadIdx.x * 4 + k;
        v[k] = j < c.table_size ? c.bucket_fill[j] : 0;
        s += v[k];
    }
    buf[threadIdx.x] = s;
    __syncthreads();
    for (int off = 1; off < 256; off <<= 1) {
        const int t = (int)threadIdx.x >= off ? buf[threadIdx.x - off] : 0;
        __syncthreads();
        buf[threadIdx.x] += t;
        __syncthreads();
    }
    int run = ((const int *)c.scan_tmp)[blockIdx.x] + buf[threadIdx.x] - s;
    for (int k = 0; k < 4; ++k) {
        const int j = base + threadIdx.x * 4 + k;
        if (j < c.table_size) {
            c.bucket_start[j] = run;
            c.bucket_fill[j] = run;   // becomes the scatter cursor
        }
        run += v[k];
    }
    if (blockIdx.x == 0 && threadIdx.x == 0) c.bucket_start[c.table_size] = c.n_surf;
}

template <typename T>
__global__ void __launch_bounds__(256) k_scatter(StepArgs<T> a, CollideArgs c) {
    if (*c.rebuild_flag == 0) return;
    T *su = (T *)c.sorted_u;
    for (int i = blockIdx.x * blockDim.x + threadIdx.x; i < c.n_surf; i += gridDim.x * blockDim.x) {
        const int pos = atomicAdd(&c.bucket_fill[c.cell_keys[i]], 1);
        const int ci = c.surf_cells[i];
        c.sorted_cell[pos] = ci;
        c.sorted_gc[pos] = c.cell_gc[i];
        c.sorted_ijk[pos] = c.cell_ijk[i];
        su[pos] = a.s_in[W_UX * a.stride + ci];
        su[c.n_surf + pos] = a.s_in[W_UY * a.stride + ci];
        su[2 * c.n_surf + pos] = a.s_in[W_UZ * a.stride + ci];
    }
}

// One workgroup serves kCandVox surface voxels with one thread per (voxel,
// neighbouring grid cell) pair: each thread scans its cell's bucket and
// appends the voxel's candidates from that cell to the voxel's list in LDS
// (an LDS counter per voxel); after a barrier every entry is written to the
// voxel's global list at its rank among the voxel's entries, so each list is
// sorted by partner cell.  Partners are distinct within a list, so the rank
// is unique.  A list that would exceed cap raises the overflow flag and
// keeps cap of its entries.
template <typename T>
__global__ void __launch_bounds__(256) k_candidates(StepArgs<T> a, CollideArgs c) {
    extern __shared__ int lds_list[];     // kCandVox x cap partner cells
    __shared__ int lds_count[kCandVox];
    if (*c.rebuild_flag == 0) return;
    const int t = threadIdx.x;
    const int v = t / 27, nb = t % 27;
    const int groups = (c.n_surf + kCandVox - 1) / kCandVox;
    // grid-stride over groups of voxels: the grid stays small for the steps
    // whose launch only finds the rebuild flag clear
    for (int grp = blockIdx.x; grp < groups; grp += gridDim.x) {
        const int i = grp * kCandVox + v;
        const bool live = v < kCandVox && i < c.n_surf;
        if (t < kCandVox) lds_count[t] = 0;
        __syncthreads();
        int ci = 0;
        if (live) {
            ci = c.surf_cells[i];
            int ix, iy, iz, cx, cy, cz;
            unpack3(c.cell_ijk[i], ix, iy, iz);
            unpack3(c.cell_gc[i], cx, cy, cz);
            const T uxi = a.s_in[W_UX * a.stride + ci], uyi = a.s_in[W_UY * a.stride + ci],
                    uzi = a.s_in[W_UZ * a.stride + ci];
            const T H = (T)c.horizon;
            const int ns = c.n_surf;
            const T *su = (const T *)c.sorted_u;
            const int tx = cx + nb % 3 - 1, ty = cy + (nb / 3) % 3 - 1, tz = cz + nb / 9 - 1;
            const int key = cell_hash(tx, ty, tz, c.table_size - 1);
            const long long want = pack3(tx, ty, tz);
            const int b0 = c.bucket_start[key], b1 = c.bucket_start[key + 1];
            // entries in groups of kGroup: the loads of a group are issued
            // together (a short last group re-reads its last entry, which is not
            // processed twice)
            for (int k0 = b0; k0 < b1; k0 += kGroup) {
                int cjg[kGroup];
                long long gcg[kGroup], ijg[kGroup];
                T uxg[kGroup], uyg[kGroup], uzg[kGroup];
    #pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    const int k = k0 + q < b1 ? k0 + q : b1 - 1;
                    cjg[q] = c.sorted_cell[k];
                    gcg[q] = c.sorted_gc[k];
                    ijg[q] = c.sorted_ijk[k];
                    uxg[q] = su[k];
                    uyg[q] = su[ns + k];
                    uzg[q] = su[2 * ns + k];
                }
    #pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    if (k0 + q >= b1) break;
                    const int cj = cjg[q];
                    if (cj == ci || gcg[q] != want) continue;   // another cell in this bucket
                    int jx, jy, jz;
                    unpack3(ijg[q], jx, jy, jz);
                    const int man = abs(jx - ix) + abs(jy - iy) + abs(jz - iz);
                    if (man <= 3) continue;
                    const T rx = T(ix - jx) * a.l + (uxi - uxg[q]);
                    const T ry = T(iy - jy) * a.l + (uyi - uyg[q]);
                    const T rz = T(iz - jz) * a.l + (uzi - uzg[q]);
                    if (!(dsqrt(rx * rx + ry * ry + rz * rz) < H)) continue;
                    const int slot = atomicAdd(&lds_count[v], 1);
                    if (slot < c.cap) lds_list[v * c.cap + slot] = cj;
                }
            }
        }
        __syncthreads();
        if (live) {
            const int count = lds_count[v];
            const int kept = count < c.cap ? count : c.cap;
            const int *mine = lds_list + v * c.cap;
            int *list = c.cand + (long long)i * c.cap;
            for (int e = nb; e < kept; e += 27) {
                const int x = mine[e];
                int rank = 0;
                for (int k = 0; k < kept; ++k) rank += mine[k] < x ? 1 : 0;
                list[rank] = x;
            }
            if (nb == 0) {
                if (count > c.cap) atomicOr(c.overflow, 1u);
                c.cand_n[i] = kept;
                // the candidate bit lives in the flags of the current step
                uint8_t *flags = const_cast<uint8_t *>(a.flags);
                uint8_t fl = flags[ci];
                fl = kept > 0 ? (uint8_t)(fl | FLAG_CAND) : (uint8_t)(fl & ~FLAG_CAND);
                flags[ci] = fl;
                if (count) atomicAdd(c.pair_count, (unsigned long long)count);
            }
        }
        __syncthreads();   // the group's lists are read before the next group reuses LDS
    }
}

__global__ void __launch_bounds__(256) k_rebuild_done(CollideArgs c) {
    if (*c.rebuild_flag == 0) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < c.table_size; j += gridDim.x * blockDim.x)
        c.bucket_fill[j] = 0;
}

__global__ void k_rebuild_clear(CollideArgs c) {
    if (*c.rebuild_flag == 0) return;
    *c.rebuild_flag = 0;
    *c.macc = 0.0;
    *c.rebuild_counter += 1;
}

template <typename T>
__global__ void __launch_bounds__(256) k_contact(StepArgs<T> a, CollideArgs c, T *cf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n_surf) return;
    const int n = c.cand_n[i];
    if (n == 0) return;
    const long long st = a.stride;
    const int ci = c.surf_cells[i];
    const uint8_t mi = a.mat[ci];
    const MatConst<T> Mi = a.mats[mi];
    const T ei = voxel_strain(a, (unsigned)ci, a.flags[ci], Mi.cte);
    const int ix = ci % a.nx, iy = (ci / a.nx) % a.ny, iz = ci / (a.nx * a.ny);
    const T ux = a.s_in[W_UX * st + ci], uy = a.s_in[W_UY * st + ci], uz = a.s_in[W_UZ * st + ci];
    const T vx = a.s_in[W_PX * st + ci] * Mi.inv_m, vy = a.s_in[W_PY * st + ci] * Mi.inv_m,
            vz = a.s_in[W_PZ * st + ci] * Mi.inv_m;
    T Fx = T(0), Fy = T(0), Fz = T(0);
    const int *list = c.cand + (long long)i * c.cap;
    for (int k = 0; k < n; ++k) {
        const int cj = list[k];
        const uint8_t mj = a.mat[cj];
        const MatConst<T> Mj = a.mats[mj];
        const int jx = cj % a.nx, jy = (cj / a.nx) % a.ny, jz = cj / (a.nx * a.ny);
        const T rx = T(ix - jx) * a.l + (ux - a.s_in[W_UX * st + cj]);
        const T ry = T(iy - jy) * a.l + (uy - a.s_in[W_UY * st + cj]);
        const T rz = T(iz - jz) * a.l + (uz - a.s_in[W_UZ * st + cj]);
        const T dist = dsqrt(rx * rx + ry * ry + rz * rz);
        const T ej = voxel_strain(a, (unsigned)cj, a.flags[cj], Mj.cte);
        const T cdist = T(0.5) * a.l * (T(1) + ei) + T(0.5) * a.l * (T(1) + ej);
        if (!(dist < cdist) || !(dist > T(0))) continue;
        const T inv = T(1) / dist;
        const T nx = rx * inv, ny = ry * inv, nz = rz * inv;
        const PairConst<T> pc = a.pairs[mi * a.n_mat + mj];
        const T vjx = a.s_in[W_PX * st + cj] * Mj.inv_m, vjy = a.s_in[W_PY * st + cj] * Mj.inv_m,
                vjz = a.s_in[W_PZ * st + cj] * Mj.inv_m;
        const T vn = (vx - vjx) * nx + (vy - vjy) * ny + (vz - vjz) * nz;
        T f = pc.kc * (cdist - dist) - pc.cc * vn;
        if (f < T(0)) f = T(0);
        Fx += f * nx; Fy += f * ny; Fz += f * nz;
    }
    cf[ci] = Fx; cf[st + ci] = Fy; cf[2 * st + ci] = Fz;
}

template <typename T>
__global__ void k_motion(StepArgs<T> a, CollideArgs c) {
    const double v = __longlong_as_double((long long)*c.vmax_bits);
    *c.vmax_bits = 0ull;
    const double m = *c.macc + v * (double)a.dt;
    *c.macc = m;
    if (c.every || 2.0 * m >= c.threshold) *c.rebuild_flag = 1u;
}

}  // namespace

size_t scan_temp_bytes(int n) { return (size_t)((n + kScanBlock - 1) / kScanBlock + 1) * sizeof(int); }

template <typename T>
hipError_t launch_rebuild(const StepArgs<T> &a, const CollideArgs &c, hipStream_t s) {
    if (c.n_surf == 0) return hipSuccess;
    Origin3 o;
    o.v[0] = a.origin[0]; o.v[1] = a.origin[1]; o.v[2] = a.origin[2];
    // grids of the per-voxel and per-bucket kernels, capped: they stride,
    // and most launches only find the rebuild flag clear
    const auto capped = [](long long n) { return (unsigned)std::min<long long>((n + 255) / 256, kCandGrid); };
    const unsigned gs = capped(c.n_surf);
    const int nblk = (c.table_size + kScanBlock - 1) / kScanBlock;
    k_keys<T><<<gs, 256, 0, s>>>(a, c, o);
    k_scan_reduce<<<nblk, 256, 0, s>>>(c);
    k_scan_blocks<<<1, 1024, 0, s>>>(c, nblk);
    k_scan_apply<<<nblk, 256, 0, s>>>(c);
    k_scatter<T><<<gs, 256, 0, s>>>(a, c);
    const int groups = (c.n_surf + kCandVox - 1) / kCandVox;
    const unsigned gc = (unsigned)(groups < kCandGrid ? groups : kCandGrid);
    k_candidates<T><<<gc, 256, (size_t)kCandVox * c.cap * sizeof(int), s>>>(a, c);
    k_rebuild_done<<<capped(c.table_size), 256, 0, s>>>(c);
    k_rebuild_clear<<<1, 1, 0, s>>>(c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_contact(const StepArgs<T> &a, const CollideArgs &c, T *contact_F, hipStream_t s) {
    if (c.n_surf == 0) return hipSuccess;
    k_contact<T><<<(unsigned)((c.n_surf + 255) / 256), 256, 0, s>>>(a, c, contact_F);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_motion_update(const StepArgs<T> &a, const CollideArgs &c, hipStream_t s) {
    k_motion<T><<<1, 1, 0, s>>>(a, c);
    return hipGetLastError();
}

template hipError_t launch_rebuild<float>(const StepArgs<float> &, const CollideArgs &, hipStream_t);
template hipError_t launch_rebuild<double>(const StepArgs<double> &, const CollideArgs &, hipStream_t);
template hipError_t launch_contact<float>(const StepArgs<float> &, const CollideArgs &, float *, hipStream_t);
template hipError_t launch_contact<double>(const StepArgs<double> &, const CollideArgs &, double *, hipStream_t);
template hipError_t launch_motion_update<float>(const StepArgs<float> &, const CollideArgs &, hipStream_t);
template hipError_t launch_motion_update<double>(const StepArgs<double> &, const CollideArgs &, hipStream_t);

}  // namespace vx
