// Linear statics on the GPU: the lattice's direct-stiffness system K x = f
// (section Validation, the "direct stiffness" column of Table 1), solved
// matrix-free by Jacobi-preconditioned conjugate gradients in FP64.
//
// x holds six degrees of freedom per voxel, displacement and rotation,
// stored as six arrays of ncell doubles.  K is never assembled: every
// face-adjacent filled pair is the 12-DOF beam element of Eq. (7) with the
// composite moduli of Eq. (1)-(2) and the section constants of Eq. (8)-(12)
// (A = l^2, I = l^4/12, J = l^4/6), laid along its lattice axis by a cyclic
// permutation of the coordinates, and each voxel gathers the forces and
// moments of its at most six elements on its own end.  Fixed and empty
// cells carry no unknowns (their entries of x, r, z, p are zero).  Dot
// products reduce per workgroup in a fixed order; the host adds the
// workgroup partials in order, so the solve is deterministic.
#include "vx_launch.hpp"

namespace vx {

namespace {

constexpr int kStaticThreads = 256;

// The six world components of DOF block k (0 = displacement, 1 = rotation)
// of cell c in a 6 x n array.
__device__ __forceinline__ void get6(const double *__restrict__ v, long long n, long long c, double u[3],
                                     double t[3]) {
    u[0] = v[c]; u[1] = v[n + c]; u[2] = v[2 * n + c];
    t[0] = v[3 * n + c]; t[1] = v[4 * n + c]; t[2] = v[5 * n + c];
}

// Constants of the element between cells with moduli E1, E2 and shear moduli
// G1, G2: a1 = Ec A / l (= b1 = 12 Ec I / l^3 for the square section),
// a2 = Gc J / l, b2 = 6 Ec I / l^2, b3 = 2 Ec I / l.
struct Elem {
    double a1, a2, b2, b3;
};

__device__ __forceinline__ Elem elem(double E1, double E2, double G1, double G2, double l) {
    const double Ec = 2.0 * E1 * E2 / (E1 + E2);
    const double Gc = 2.0 * G1 * G2 / (G1 + G2);
    Elem e;
    e.a1 = Ec * l;
    e.a2 = Gc * l * l * l / 6.0;
    e.b2 = Ec * l * l / 2.0;
    e.b3 = Ec * l * l * l / 6.0;
    return e;
}

// Whether cell c has unknowns, and the neighbour of c one step along axis
// ax in direction dir (+1 / -1), or -1.
__device__ __forceinline__ bool active(const StaticArgs &s, long long c) {
    return s.mat[c] != 0 && s.fixed[c] == 0;
}

__device__ __forceinline__ long long neighbour(const StaticArgs &s, long long c, int ax, int dir) {
    const int idx[3] = {(int)(c % s.nx), (int)((c / s.nx) % s.ny), (int)(c / ((long long)s.nx * s.ny))};
    const int dim[3] = {s.nx, s.ny, s.nz};
    const long long step[3] = {1, s.nx, (long long)s.nx * s.ny};
    const int k = idx[ax] + dir;
    if (k < 0 || k >= dim[ax]) return -1;
    const long long cn = c + dir * step[ax];
    return s.mat[cn] != 0 ? cn : -1;
}

// q = K p on the cells with unknowns (0 elsewhere), and the workgroup's
// partial of p . q.
__global__ void __launch_bounds__(kStaticThreads) k_static_apply(StaticArgs s, const double *__restrict__ p,
                                                                 double *__restrict__ q, double *partials) {
    __shared__ double red[kStaticThreads];
    const long long c = (long long)blockIdx.x * kStaticThreads + threadIdx.x;
    const long long n = s.n;
    double acc = 0.0;
    if (c < n && active(s, c)) {
        double u0[3], t0[3];
        get6(p, n, c, u0, t0);
        double F[3] = {0.0, 0.0, 0.0}, M[3] = {0.0, 0.0, 0.0};
        for (int ax = 0; ax < 3; ++ax) {
            for (int dir = 1; dir >= -1; dir -= 2) {
                const long long cn = neighbour(s, c, ax, dir);
                if (cn < 0) continue;
                double un[3], tn[3];
                get6(p, n, cn, un, tn);
                const Elem e = elem(s.E[c], s.E[cn], s.G[c], s.G[cn], s.l);
                // end 1 is the lower cell of the pair; local axis i is world
                // axis (ax + i) mod 3
                const double *u1 = dir > 0 ? u0 : un, *t1 = dir > 0 ? t0 : tn;
                const double *u2 = dir > 0 ? un : u0, *t2 = dir > 0 ? tn : t0;
                const int i0 = ax, i1 = (ax + 1) % 3, i2 = (ax + 2) % 3;
                const double dX = u1[i0] - u2[i0], dY = u1[i1] - u2[i1], dZ = u1[i2] - u2[i2];
                const double fX = e.a1 * dX;
                const double fY = e.a1 * dY + e.b2 * (t1[i2] + t2[i2]);
                const double fZ = e.a1 * dZ - e.b2 * (t1[i1] + t2[i1]);
                const double mX = e.a2 * (t1[i0] - t2[i0]);
                double mY, mZ;
                if (dir > 0) {   // this cell is end 1
                    mY = -e.b2 * dZ + 2.0 * e.b3 * t1[i1] + e.b3 * t2[i1];
                    mZ = e.b2 * dY + 2.0 * e.b3 * t1[i2] + e.b3 * t2[i2];
                    F[i0] += fX; F[i1] += fY; F[i2] += fZ;
                    M[i0] += mX; M[i1] += mY; M[i2] += mZ;
                } else {         // end 2: forces and torsion opposite
                    mY = -e.b2 * dZ + e.b3 * t1[i1] + 2.0 * e.b3 * t2[i1];
                    mZ = e.b2 * dY + e.b3 * t1[i2] + 2.0 * e.b3 * t2[i2];
                    F[i0] -= fX; F[i1] -= fY; F[i2] -= fZ;
                    M[i0] -= mX; M[i1] += mY; M[i2] += mZ;
                }
            }
        }
        for (int k = 0; k < 3; ++k) {
            q[k * n + c] = F[k];
            q[(3 + k) * n + c] = M[k];
            acc += u0[k] * F[k] + t0[k] * M[k];
        }
    } else if (c < n) {
        for (int k = 0; k < 6; ++k) q[k * n + c] = 0.0;
    }
    red[threadIdx.x] = acc;
    __syncthreads();
    for (int h = kStaticThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) red[threadIdx.x] += red[threadIdx.x + h];
        __syncthreads();
    }
    if (threadIdx.x == 0) partials[blockIdx.x] = red[0];
}

// Jacobi preconditioner: the diagonal of K per unknown (a1, b1 = a1, b1,
// a2, 2 b3, 2 b3 in each element's local order, the same at both ends).
__global__ void __launch_bounds__(kStaticThreads) k_static_diag(StaticArgs s, double *__restrict__ diag) {
    const long long c = (long long)blockIdx.x * kStaticThreads + threadIdx.x;
    const long long n = s.n;
    if (c >= n) return;
    double d[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
    if (active(s, c)) {
        for (int ax = 0; ax < 3; ++ax)
            for (int dir = 1; dir >= -1; dir -= 2) {
                const long long cn = neighbour(s, c, ax, dir);
                if (cn < 0) continue;
                const Elem e = elem(s.E[c], s.E[cn], s.G[c], s.G[cn], s.l);
                const int i0 = ax, i1 = (ax + 1) % 3, i2 = (ax + 2) % 3;
                d[i0] += e.a1; d[i1] += e.a1; d[i2] += e.a1;
                d[3 + i0] += e.a2; d[3 + i1] += 2.0 * e.b3; d[3 + i2] += 2.0 * e.b3;
            }
    }
    // cells without unknowns (or a voxel with no bond) get 1: their r is 0
    for (int k = 0; k < 6; ++k) diag[k * n + c] = d[k] > 0.0 ? d[k] : 1.0;
}

// Start: x = 0, r = f on the unknowns, z = r / diag, p = z; partials of
// r . z (first half) and f . f (second half).
__global__ void __launch_bounds__(kStaticThreads) k_static_start(StaticArgs s, const double *__restrict__ f,
                                                                 const double *__restrict__ diag, double *x,
                                                                 double *r, double *z, double *p,
                                                                 double *partials) {
    __shared__ double red[2][kStaticThreads];
    const long long c = (long long)blockIdx.x * kStaticThreads + threadIdx.x;
    const long long n = s.n;
    double rz = 0.0, ff = 0.0;
    if (c < n) {
        const bool a = active(s, c);
        for (int k = 0; k < 6; ++k) {
            const double rk = a ? f[k * n + c] : 0.0;
            const double zk = rk / diag[k * n + c];
            x[k * n + c] = 0.0;
            r[k * n + c] = rk;
            z[k * n + c] = zk;
            p[k * n + c] = zk;
            rz += rk * zk;
            ff += rk * rk;
        }
    }
    red[0][threadIdx.x] = rz;
    red[1][threadIdx.x] = ff;
    __syncthreads();
    for (int h = kStaticThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0];
        partials[2 * blockIdx.x + 1] = red[1][0];
    }
}

// x += alpha p, r -= alpha q, z = r / diag; partials of r . z and r . r.
__global__ void __launch_bounds__(kStaticThreads) k_static_step(StaticArgs s, double alpha,
                                                                const double *__restrict__ p,
                                                                const double *__restrict__ q,
                                                                const double *__restrict__ diag, double *x,
                                                                double *r, double *z, double *partials) {
    __shared__ double red[2][kStaticThreads];
    const long long c = (long long)blockIdx.x * kStaticThreads + threadIdx.x;
    const long long n = s.n;
    double rz = 0.0, rr = 0.0;
    if (c < n) {
        for (int k = 0; k < 6; ++k) {
            const long long i = k * n + c;
            x[i] += alpha * p[i];
            const double rk = r[i] - alpha * q[i];
            const double zk = rk / diag[i];
            r[i] = rk;
            z[i] = zk;
            rz += rk * zk;
            rr += rk * rk;
        }
    }
    red[0][threadIdx.x] = rz;
    red[1][threadIdx.x] = rr;
    __syncthreads();
    for (int h = kStaticThreads / 2; h > 0; h >>= 1) {
        if ((int)threadIdx.x < h) {
            red[0][threadIdx.x] += red[0][threadIdx.x + h];
            red[1][threadIdx.x] += red[1][threadIdx.x + h];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        partials[2 * blockIdx.x] = red[0][0];
        partials[2 * blockIdx.x + 1] = red[1][0];
    }
}

// p = z + beta p.
__global__ void __launch_bounds__(kStaticThreads) k_static_dir(long long n6, double beta,
                                                               const double *__restrict__ z, double *p) {
    const long long i = (long long)blockIdx.x * kStaticThreads + threadIdx.x;
    if (i < n6) p[i] = z[i] + beta * p[i];
}

}  // namespace

int static_blocks(long long ncell) { return (int)((ncell + kStaticThreads - 1) / kStaticThreads); }

hipError_t launch_static_diag(const StaticArgs &s, double *diag, hipStream_t st) {
    k_static_diag<<<static_blocks(s.n), kStaticThreads, 0, st>>>(s, diag);
    return hipGetLastError();
}

hipError_t launch_static_start(const StaticArgs &s, const double *f, const double *diag, double *x, double *r,
                               double *z, double *p, double *partials, hipStream_t st) {
    k_static_start<<<static_blocks(s.n), kStaticThreads, 0, st>>>(s, f, diag, x, r, z, p, partials);
    return hipGetLastError();
}

hipError_t launch_static_apply(const StaticArgs &s, const double *p, double *q, double *partials, hipStream_t st) {
    k_static_apply<<<static_blocks(s.n), kStaticThreads, 0, st>>>(s, p, q, partials);
    return hipGetLastError();
}

hipError_t launch_static_step(const StaticArgs &s, double alpha, const double *p, const double *q,
                              const double *diag, double *x, double *r, double *z, double *partials,
                              hipStream_t st) {
    k_static_step<<<static_blocks(s.n), kStaticThreads, 0, st>>>(s, alpha, p, q, diag, x, r, z, partials);
    return hipGetLastError();
}

hipError_t launch_static_dir(long long ncell, double beta, const double *z, double *p, hipStream_t st) {
    const long long n6 = 6 * ncell;
    k_static_dir<<<(unsigned)((n6 + kStaticThreads - 1) / kStaticThreads), kStaticThreads, 0, st>>>(n6, beta, z, p);
    return hipGetLastError();
}

}  // namespace vx
