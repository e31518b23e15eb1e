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

// Separation D_i - D_j of two listed voxels from their rest indices within
// their objects, the objects' origins and their displacements.  Within one
// object the rest offset is an exact multiple of l.
template <typename T>
__device__ __forceinline__ void separation(const CollideArgs &c, T l, int oi, int ix, int iy, int iz, int oj, int jx,
                                           int jy, int jz, T dux, T duy, T duz, T &rx, T &ry, T &rz) {
    if (oi == oj) {
        rx = T(ix - jx) * l + dux;
        ry = T(iy - jy) * l + duy;
        rz = T(iz - jz) * l + duz;
    } else {
        const double *a = c.obj_origin + 3 * oi, *b = c.obj_origin + 3 * oj;
        const double L = (double)l;
        rx = (T)((a[0] - b[0]) + (double)(ix - jx) * L) + dux;
        ry = (T)((a[1] - b[1]) + (double)(iy - jy) * L) + duy;
        rz = (T)((a[2] - b[2]) + (double)(iz - jz) * L) + duz;
    }
}

// Surface voxels per workgroup of the candidate search (27 threads each),
// and the largest grid of the rebuild kernels (they stride over their work).
constexpr int kCandVox = 9;
constexpr int kCandGrid = 512;
// bucket entries whose loads the candidate search issues together
constexpr int kGroup = 4;

// Grid cell and hash key of every listed voxel; bucket counts and the
// counts per scan block.  The last workgroup to finish turns the block
// counts into their exclusive prefix.
template <typename T>
__global__ void __launch_bounds__(256) k_keys(StepArgs<T> a, CollideArgs c, int nblk) {
    __shared__ int last;
    __shared__ int part[256];
    if (*c.rebuild_flag == 0) return;
    const int first = blockIdx.x * blockDim.x + threadIdx.x;
    if (first == 0) *c.pair_count = 0ull;
    const double H = c.horizon;
    for (int i = first; i < c.n_surf; i += gridDim.x * blockDim.x) {
        const int ci = c.surf_cells[i], ob = c.surf_obj[i];
        int ix, iy, iz;
        unpack3(c.surf_ijk[i], ix, iy, iz);
        const double *o = c.obj_origin + 3 * ob;
        // world position in the state precision: origin + (index + 1/2) l + u
        const T x = (T)o[0] + (T(ix) + T(0.5)) * a.l + a.s_in[W_UX * a.stride + ci];
        const T y = (T)o[1] + (T(iy) + T(0.5)) * a.l + a.s_in[W_UY * a.stride + ci];
        const T z = (T)o[2] + (T(iz) + T(0.5)) * a.l + a.s_in[W_UZ * a.stride + ci];
        const int cx = (int)floor((double)x / H), cy = (int)floor((double)y / H), cz = (int)floor((double)z / H);
        const int key = cell_hash(cx, cy, cz, c.table_size - 1);
        c.cell_keys[i] = key;
        c.cell_gc[i] = pack3(cx, cy, cz);
        atomicAdd(&c.bucket_fill[key], 1);
        atomicAdd(&c.block_sum[key / kScanBlock], 1);
    }
    __threadfence();
    __syncthreads();
    if (threadIdx.x == 0) last = atomicAdd(c.done, 1u) == gridDim.x - 1;
    __syncthreads();
    if (!last) return;
    __threadfence();
    // exclusive prefix of the block counts, 256 blocks at a time
    int carry = 0;
    for (int base = 0; base < nblk; base += 256) {
        const int j = base + (int)threadIdx.x;
        const int v = j < nblk ? atomicAdd(&c.block_sum[j], 0) : 0;
        part[threadIdx.x] = v;
        __syncthreads();
        for (int off = 1; off < 256; off <<= 1) {
            const int t = (int)threadIdx.x >= off ? part[threadIdx.x - off] : 0;
            __syncthreads();
            part[threadIdx.x] += t;
            __syncthreads();
        }
        if (j < nblk) c.block_sum[j] = carry + part[threadIdx.x] - v;
        carry += part[255];
        __syncthreads();
    }
    if (threadIdx.x == 0) *c.done = 0u;
}

// Bucket starts: each scan block's exclusive prefix of its own counts plus
// the block's offset; the starts become the scatter cursors.
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
    int run = c.block_sum[blockIdx.x] + buf[threadIdx.x] - s;
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
        c.sorted_idx[pos] = i;
        c.sorted_gc[pos] = c.cell_gc[i];
        c.sorted_ijk[pos] = c.surf_ijk[i];
        c.sorted_obj[pos] = c.surf_obj[i];
        su[pos] = a.s_in[W_UX * a.stride + ci];
        su[c.n_surf + pos] = a.s_in[W_UY * a.stride + ci];
        su[2 * c.n_surf + pos] = a.s_in[W_UZ * a.stride + ci];
    }
}

// One workgroup serves kCandVox listed voxels with one thread per (voxel,
// neighbouring grid cell) pair: each thread scans its cell's bucket and
// appends the voxel's candidates from that cell to the voxel's list in LDS
// (an LDS counter per voxel); after a barrier every entry is written to the
// voxel's global list at its rank among the voxel's entries, so each list is
// sorted by partner.  Partners are distinct within a list, so the rank is
// unique.  A list that would exceed cap raises the overflow flag and keeps
// cap of its entries.  Pairs within one object closer than Manhattan
// distance 4 in rest indices are excluded.  The launch also clears the
// bucket counts and block sums for the next rebuild (nothing here reads
// them).
template <typename T>
__global__ void __launch_bounds__(256) k_candidates(StepArgs<T> a, CollideArgs c, int nblk) {
    extern __shared__ int lds_list[];     // kCandVox x cap partner indices
    __shared__ int lds_count[kCandVox];
    if (*c.rebuild_flag == 0) return;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < c.table_size; j += gridDim.x * blockDim.x)
        c.bucket_fill[j] = 0;
    for (int j = blockIdx.x * blockDim.x + threadIdx.x; j < nblk; j += gridDim.x * blockDim.x) c.block_sum[j] = 0;
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
            const int oi = c.surf_obj[i];
            int ix, iy, iz, cx, cy, cz;
            unpack3(c.surf_ijk[i], ix, iy, iz);
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
                int jg[kGroup], og[kGroup];
                long long gcg[kGroup], ijg[kGroup];
                T uxg[kGroup], uyg[kGroup], uzg[kGroup];
    #pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    const int k = k0 + q < b1 ? k0 + q : b1 - 1;
                    jg[q] = c.sorted_idx[k];
                    gcg[q] = c.sorted_gc[k];
                    ijg[q] = c.sorted_ijk[k];
                    og[q] = c.sorted_obj[k];
                    uxg[q] = su[k];
                    uyg[q] = su[ns + k];
                    uzg[q] = su[2 * ns + k];
                }
    #pragma unroll
                for (int q = 0; q < kGroup; ++q) {
                    if (k0 + q >= b1) break;
                    const int j = jg[q];
                    if (j == i || gcg[q] != want) continue;   // itself, or another cell in this bucket
                    int jx, jy, jz;
                    unpack3(ijg[q], jx, jy, jz);
                    if (og[q] == oi && abs(jx - ix) + abs(jy - iy) + abs(jz - iz) <= 3) continue;
                    T rx, ry, rz;
                    separation(c, a.l, oi, ix, iy, iz, og[q], jx, jy, jz, uxi - uxg[q], uyi - uyg[q], uzi - uzg[q],
                               rx, ry, rz);
                    if (!(dsqrt(rx * rx + ry * ry + rz * rz) < H)) continue;
                    const int slot = atomicAdd(&lds_count[v], 1);
                    if (slot < c.cap) lds_list[v * c.cap + slot] = j;
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

// Contact constants of a pair (the bond's translational stiffness and the
// collision damping coefficient over the lighter mass, as the host tables
// hold them per material pair), from the palette, or in parameter mode from
// the two cells' own moduli and masses in the same order of operations.
template <typename T>
struct ContactK {
    T kc, cc;
};

template <typename T>
__device__ __forceinline__ ContactK<T> contact_k(const StepArgs<T> &a, unsigned ci, unsigned cj, uint8_t mi,
                                                 uint8_t mj, const MatConst<T> &Mi, const MatConst<T> &Mj) {
    ContactK<T> k;
    if (a.E_cell) {
        const T Ei = a.E_cell[ci], Ej = a.E_cell[cj];
        k.kc = (T(2) * Ei * Ej / (Ei + Ej)) * a.l;
        const T mmin = Mi.m < Mj.m ? Mi.m : Mj.m;
        k.cc = T(2) * a.zeta_col * dsqrt(mmin * k.kc);
    } else {
        const PairConst<T> pc = a.pairs[mi * a.n_mat + mj];
        k.kc = pc.kc;
        k.cc = pc.cc;
    }
    return k;
}

template <typename T>
__global__ void __launch_bounds__(256) k_contact(StepArgs<T> a, CollideArgs c, T *cf) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n_surf) return;
    const int n = c.cand_n[i];
    if (n == 0) return;
    const long long st = a.stride;
    const int ci = c.surf_cells[i], oi = c.surf_obj[i];
    const uint8_t mi = a.mat[ci];
    const MatConst<T> Mi = mat_at(a, ci, mi);
    const T ei = voxel_strain(a, (unsigned)ci, a.flags[ci], Mi.cte);
    int ix, iy, iz;
    unpack3(c.surf_ijk[i], ix, iy, iz);
    const T ux = a.s_in[W_UX * st + ci], uy = a.s_in[W_UY * st + ci], uz = a.s_in[W_UZ * st + ci];
    const T vx = a.s_in[W_PX * st + ci] * Mi.inv_m, vy = a.s_in[W_PY * st + ci] * Mi.inv_m,
            vz = a.s_in[W_PZ * st + ci] * Mi.inv_m;
    T Fx = T(0), Fy = T(0), Fz = T(0);
    const int *list = c.cand + (long long)i * c.cap;
    for (int k = 0; k < n; ++k) {
        const int j = list[k];
        const int cj = c.surf_cells[j], oj = c.surf_obj[j];
        const uint8_t mj = a.mat[cj];
        const MatConst<T> Mj = mat_at(a, cj, mj);
        int jx, jy, jz;
        unpack3(c.surf_ijk[j], jx, jy, jz);
        T rx, ry, rz;
        separation(c, a.l, oi, ix, iy, iz, oj, jx, jy, jz, ux - a.s_in[W_UX * st + cj], uy - a.s_in[W_UY * st + cj],
                   uz - a.s_in[W_UZ * st + cj], rx, ry, rz);
        const T dist = dsqrt(rx * rx + ry * ry + rz * rz);
        const T ej = voxel_strain(a, (unsigned)cj, a.flags[cj], Mj.cte);
        const T cdist = T(0.5) * a.l * (T(1) + ei) + T(0.5) * a.l * (T(1) + ej);
        if (!(dist < cdist) || !(dist > T(0))) continue;
        const T inv = T(1) / dist;
        const T nx = rx * inv, ny = ry * inv, nz = rz * inv;
        const ContactK<T> pc = contact_k(a, (unsigned)ci, (unsigned)cj, mi, mj, Mi, Mj);
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
    const unsigned rebuilt = motion_update(c.scalars, (double)a.dt);
    if (c.rlog) *c.rlog = rebuilt ? 1 : 0;
}

__global__ void k_force_rebuild(CollideArgs c) { *c.rebuild_flag = 1u; }

// Reverse of one pair term f n of a contact force, with f = kc (cdist -
// dist) - cc vn > 0, n = r / dist, vn = dv . n, given the adjoint lam of the
// force: the adjoints of r, dv, cdist, kc and cc.
template <typename T>
struct PairAdj {
    T r[3], dv[3], cdist, kc, cc;
};

template <typename T>
__device__ __forceinline__ PairAdj<T> pair_vjp(const T lam[3], const T n[3], const T dv[3], T f, T inv, T kc, T cc,
                                               T cdist, T dist, T vn) {
    PairAdj<T> g;
    const T gf = lam[0] * n[0] + lam[1] * n[1] + lam[2] * n[2];
    T gn[3];
    for (int k = 0; k < 3; ++k) gn[k] = f * lam[k] - gf * cc * dv[k];
    const T gnn = gn[0] * n[0] + gn[1] * n[1] + gn[2] * n[2];
    const T gdist = -gf * kc;
    for (int k = 0; k < 3; ++k) {
        g.r[k] = (gn[k] - gnn * n[k]) * inv + gdist * n[k];
        g.dv[k] = -gf * cc * n[k];
    }
    g.cdist = gf * kc;
    g.kc = gf * (cdist - dist);
    g.cc = -gf * vn;
    return g;
}

// Reverse of the contact forces of one step, per listed voxel i: the terms
// of i's own force (adjoint: i's bond-sum force adjoint, which the update
// adds the contact force to) and of each partner's force on which i's state
// acts (the partner's adjoint), gathered without atomics from i's own list
// (the lists are symmetric).  Adds to the adjoint of i's displacement and
// momentum and to the update's adjoints of i's strain, modulus and mass;
// runs between the update's and the bonds' reverse kernels of the step.
template <typename T>
__global__ void __launch_bounds__(256) k_adj_contact(StepArgs<T> a, CollideArgs c, AdjArgs<T> g) {
    const int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= c.n_surf) return;
    const int n = c.cand_n[i];
    if (n == 0) return;
    const long long st = a.stride;
    const int ci = c.surf_cells[i], oi = c.surf_obj[i];
    const uint8_t mi = a.mat[ci];
    const MatConst<T> Mi = mat_at(a, ci, mi);
    const T ei = voxel_strain(a, (unsigned)ci, a.flags[ci], Mi.cte);
    int ix, iy, iz;
    unpack3(c.surf_ijk[i], ix, iy, iz);
    const T ui[3] = {a.s_in[W_UX * st + ci], a.s_in[W_UY * st + ci], a.s_in[W_UZ * st + ci]};
    const T Pi[3] = {a.s_in[W_PX * st + ci], a.s_in[W_PY * st + ci], a.s_in[W_PZ * st + ci]};
    const T vi[3] = {Pi[0] * Mi.inv_m, Pi[1] * Mi.inv_m, Pi[2] * Mi.inv_m};
    const T lami[3] = {g.gfm[ci], g.gfm[st + ci], g.gfm[2 * st + ci]};
    T gu[3] = {T(0), T(0), T(0)}, gv[3] = {T(0), T(0), T(0)};
    T geps = T(0), gE = T(0), gm = T(0);
    const int *list = c.cand + (long long)i * c.cap;
    for (int k = 0; k < n; ++k) {
        const int j = list[k];
        const int cj = c.surf_cells[j], oj = c.surf_obj[j];
        const uint8_t mj = a.mat[cj];
        const MatConst<T> Mj = mat_at(a, cj, mj);
        int jx, jy, jz;
        unpack3(c.surf_ijk[j], jx, jy, jz);
        T r[3];
        separation(c, a.l, oi, ix, iy, iz, oj, jx, jy, jz, ui[0] - a.s_in[W_UX * st + cj],
                   ui[1] - a.s_in[W_UY * st + cj], ui[2] - a.s_in[W_UZ * st + cj], r[0], r[1], r[2]);
        const T dist = dsqrt(r[0] * r[0] + r[1] * r[1] + r[2] * r[2]);
        const T ej = voxel_strain(a, (unsigned)cj, a.flags[cj], Mj.cte);
        const T cdist = T(0.5) * a.l * (T(1) + ei) + T(0.5) * a.l * (T(1) + ej);
        if (!(dist < cdist) || !(dist > T(0))) continue;
        const T inv = T(1) / dist;
        const T nv[3] = {r[0] * inv, r[1] * inv, r[2] * inv};
        const ContactK<T> K = contact_k(a, (unsigned)ci, (unsigned)cj, mi, mj, Mi, Mj);
        const T Pj[3] = {a.s_in[W_PX * st + cj], a.s_in[W_PY * st + cj], a.s_in[W_PZ * st + cj]};
        const T dv[3] = {vi[0] - Pj[0] * Mj.inv_m, vi[1] - Pj[1] * Mj.inv_m, vi[2] - Pj[2] * Mj.inv_m};
        const T vn = dv[0] * nv[0] + dv[1] * nv[1] + dv[2] * nv[2];
        const T f = K.kc * (cdist - dist) - K.cc * vn;
        if (!(f > T(0))) continue;
        // i's own force: pair (i, j), r = D_i - D_j, dv = v_i - v_j
        const PairAdj<T> A = pair_vjp(lami, nv, dv, f, inv, K.kc, K.cc, cdist, dist, vn);
        // j's force on which i acts: pair (j, i), r' = -r, dv' = -dv, the
        // same f and vn
        const T lamj[3] = {g.gfm[cj], g.gfm[st + cj], g.gfm[2 * st + cj]};
        const T nm[3] = {-nv[0], -nv[1], -nv[2]}, dvm[3] = {-dv[0], -dv[1], -dv[2]};
        const PairAdj<T> B = pair_vjp(lamj, nm, dvm, f, inv, K.kc, K.cc, cdist, dist, vn);
        for (int q = 0; q < 3; ++q) {
            gu[q] += A.r[q] - B.r[q];
            gv[q] += A.dv[q] - B.dv[q];
        }
        geps += (A.cdist + B.cdist) * (T(0.5) * a.l);
        if (a.E_cell) {
            // kc = E_c l with E_c = 2 E_i E_j / (E_i + E_j); cc = 2 zeta
            // sqrt(m_min kc)
            const T Ei = a.E_cell[ci], Ej = a.E_cell[cj], s = Ei + Ej;
            const T gkc = (A.kc + B.kc) + (A.cc + B.cc) * K.cc / (T(2) * K.kc);
            gE += gkc * a.l * (T(2) * Ej * Ej / (s * s));
            const T mmin = Mi.m < Mj.m ? Mi.m : Mj.m;
            const T dcc_dm = K.cc / (T(2) * mmin);
            // both forces of the pair take the same smaller mass; on a
            // tie each voxel takes half of its derivative
            const T wi = Mi.m < Mj.m ? T(1) : (Mj.m < Mi.m ? T(0) : T(0.5));
            gm += (A.cc + B.cc) * dcc_dm * wi;
        }
    }
    // v_i = P_i / m_i
    const T ginv_m = gv[0] * Pi[0] + gv[1] * Pi[1] + gv[2] * Pi[2];
    gm -= ginv_m * Mi.inv_m * Mi.inv_m;
    T *lo = g.lam_out;
    lo[W_UX * st + ci] += gu[0]; lo[W_UY * st + ci] += gu[1]; lo[W_UZ * st + ci] += gu[2];
    lo[W_PX * st + ci] += gv[0] * Mi.inv_m; lo[W_PY * st + ci] += gv[1] * Mi.inv_m;
    lo[W_PZ * st + ci] += gv[2] * Mi.inv_m;
    g.gloc[ci] += geps;
    g.gloc[st + ci] += gE;
    g.gloc[2 * st + ci] += gm;
}

}  // namespace

int scan_blocks(int n) { return (n + kScanBlock - 1) / kScanBlock; }

template <typename T>
hipError_t launch_rebuild(const StepArgs<T> &a, const CollideArgs &c, hipStream_t s) {
    if (c.n_surf == 0) return hipSuccess;
    // grids of the per-voxel kernels, capped: they stride, and most
    // launches only find the rebuild flag clear
    const auto capped = [](long long n) { return (unsigned)std::min<long long>((n + 255) / 256, kCandGrid); };
    const unsigned gs = capped(c.n_surf);
    const int nblk = scan_blocks(c.table_size);
    k_keys<T><<<gs, 256, 0, s>>>(a, c, nblk);
    k_scan_apply<<<nblk, 256, 0, s>>>(c);
    k_scatter<T><<<gs, 256, 0, s>>>(a, c);
    const int groups = (c.n_surf + kCandVox - 1) / kCandVox;
    const unsigned gc = (unsigned)(groups < kCandGrid ? groups : kCandGrid);
    k_candidates<T><<<gc, 256, (size_t)kCandVox * c.cap * sizeof(int), s>>>(a, c, nblk);
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

hipError_t launch_force_rebuild(const CollideArgs &c, hipStream_t s) {
    k_force_rebuild<<<1, 1, 0, s>>>(c);
    return hipGetLastError();
}

template <typename T>
hipError_t launch_adjoint_contact(const StepArgs<T> &a, const CollideArgs &c, const AdjArgs<T> &g, hipStream_t s) {
    if (c.n_surf == 0) return hipSuccess;
    k_adj_contact<T><<<(unsigned)((c.n_surf + 255) / 256), 256, 0, s>>>(a, c, g);
    return hipGetLastError();
}

template hipError_t launch_rebuild<float>(const StepArgs<float> &, const CollideArgs &, hipStream_t);
template hipError_t launch_rebuild<double>(const StepArgs<double> &, const CollideArgs &, hipStream_t);
template hipError_t launch_contact<float>(const StepArgs<float> &, const CollideArgs &, float *, hipStream_t);
template hipError_t launch_contact<double>(const StepArgs<double> &, const CollideArgs &, double *, hipStream_t);
template hipError_t launch_motion_update<float>(const StepArgs<float> &, const CollideArgs &, hipStream_t);
template hipError_t launch_adjoint_contact<float>(const StepArgs<float> &, const CollideArgs &,
                                                  const AdjArgs<float> &, hipStream_t);
template hipError_t launch_adjoint_contact<double>(const StepArgs<double> &, const CollideArgs &,
                                                   const AdjArgs<double> &, hipStream_t);
template hipError_t launch_motion_update<double>(const StepArgs<double> &, const CollideArgs &, hipStream_t);

}  // namespace vx
