// Host side of the linear static solve (vx_static_workspace_bytes,
// vx_static_solve, vx_static_solve_noalloc): workspace layout, upload of the
// per-cell moduli, the clamp mask and the load, and the conjugate-gradient
// loop, whose scalars come from the kernels' per-workgroup partials added
// in order.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <mutex>
#include <vector>

#include "vx_host.hpp"
#include "vx_sim.hpp"

namespace {

struct StaticLayout {
    uint64_t E, G, fixed, f, x, r, z, p, q, diag, partials, total;
};

StaticLayout static_layout(const vx_sim *h) {
    const uint64_t n = (uint64_t)h->ncell;
    const uint64_t v6 = 6 * n * 8;
    StaticLayout L{};
    uint64_t off = 0;
    auto take = [&](uint64_t bytes) { uint64_t o = off; off = align_up(off + std::max<uint64_t>(bytes, 1)); return o; };
    L.E = take(n * 8);
    L.G = take(n * 8);
    L.fixed = take(n);
    L.f = take(v6);
    L.x = take(v6);
    L.r = take(v6);
    L.z = take(v6);
    L.p = take(v6);
    L.q = take(v6);
    L.diag = take(v6);
    L.partials = take((uint64_t)2 * static_blocks((long long)n) * 8);
    L.total = off;
    return L;
}

}  // namespace

// Workspace of vx_static_solve_noalloc: one fixed device array, so that the
// call needs no allocation.  Every device the library runs on holds its own
// copy until the process ends.  In host code the array's name is not a
// device address: kernels get the address hipGetSymbolAddress returns for
// the device (scratch_ptr).
constexpr uint64_t kStaticScratchBytes = 64ull << 20;
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

namespace {

constexpr int kMaxDevices = 64;
std::mutex scratch_mu;
void *scratch_dev[kMaxDevices] = {};

// Address of device dev's scratch, looked up once per device with that
// device current.
hipError_t scratch_ptr(int dev, void **out) {
    if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
    std::lock_guard<std::mutex> lock(scratch_mu);
    if (!scratch_dev[dev]) {
        int prev = 0;
        hipError_t e = hipGetDevice(&prev);
        if (e != hipSuccess) return e;
        if (prev != dev && (e = hipSetDevice(dev)) != hipSuccess) return e;
        void *p = nullptr;
        e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (prev != dev) {
            const hipError_t e2 = hipSetDevice(prev);
            if (e == hipSuccess) e = e2;
        }
        if (e != hipSuccess) return e;
        scratch_dev[dev] = p;
    }
    *out = scratch_dev[dev];
    return hipSuccess;
}

// The solve itself on a workspace w laid out by static_layout(h).
int static_solve(vx_sim *h, char *w, const double *F, double rel_tol, int32_t max_iter, double *u,
                 double *theta, int32_t *iters, double *rel_residual);

}  // namespace

extern "C" {

int vx_static_workspace_bytes(vx_handle h, uint64_t *bytes) {
    VX_TRY
    if (!h || !bytes) return VX_EINVAL;
    *bytes = static_layout(h).total;
    return VX_OK;
    VX_CATCH(h)
}

int vx_static_solve(vx_handle h, void *work, uint64_t work_bytes, const double *F, double rel_tol,
                    int32_t max_iter, double *u, double *theta, int32_t *iters, double *rel_residual) {
    VX_TRY
    if (!h || !F || !(rel_tol > 0.0) || max_iter < 1) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_static_solve before vx_bind_workspace");
    const StaticLayout L = static_layout(h);
    if (!work || work_bytes < L.total) return fail(h, VX_EINVAL, "static workspace too small");
    if (((uintptr_t)work) % kAlign) return fail(h, VX_EINVAL, "static workspace not 256-byte aligned");
    return static_solve(h, (char *)work, F, rel_tol, max_iter, u, theta, iters, rel_residual);
    VX_CATCH(h)
}

int vx_static_solve_noalloc(vx_handle h, const double *F, double rel_tol, int32_t max_iter, double *u,
                            double *theta, int32_t *iters, double *rel_residual) {
    VX_TRY
    if (!h || !F || !(rel_tol > 0.0) || max_iter < 1) return VX_EINVAL;
    if (!h->bound) return fail(h, VX_ESTATE, "vx_static_solve_noalloc before vx_bind_workspace");
    const StaticLayout L = static_layout(h);
    if (L.total > kStaticScratchBytes)
        return fail(h, VX_EINVAL, "lattice too large for vx_static_solve_noalloc: its workspace needs " +
                                      std::to_string(L.total) + " bytes, the fixed scratch holds " +
                                      std::to_string(kStaticScratchBytes));
    // the scratch of the device the handle's stream runs on
    int dev = 0;
    if (h->stream) {
        HIP_OK(h, hipStreamGetDevice(h->stream, &dev));
    } else {
        HIP_OK(h, hipGetDevice(&dev));
    }
    void *w = nullptr;
    HIP_OK(h, scratch_ptr(dev, &w));
    return static_solve(h, (char *)w, F, rel_tol, max_iter, u, theta, iters, rel_residual);
    VX_CATCH(h)
}

}  // extern "C"

namespace {

int static_solve(vx_sim *h, char *w, const double *F, double rel_tol, int32_t max_iter, double *u,
                 double *theta, int32_t *iters, double *rel_residual) {
    const StaticLayout L = static_layout(h);
    const long long n = h->ncell;
    for (long long i = 0; i < 3 * n; ++i)
        if (!std::isfinite(F[i])) return fail(h, VX_EINVAL, "non-finite force");
    hipStream_t s = h->stream;
    // per-cell moduli as the step uses them (palette, or the cell's own in
    // parameter mode); shear modulus from the material's Poisson ratio
    std::vector<double> E(n, 0.0), G(n, 0.0), f(6 * n, 0.0);
    std::vector<uint8_t> fixed(n, 0);
    for (long long c = 0; c < n; ++c) {
        const int m = h->grid[c];
        if (!m) continue;
        E[c] = h->has_E ? h->E_cell[c] : h->pal[m].E;
        G[c] = E[c] / (2.0 * (1.0 + h->pal[m].nu));
        fixed[c] = (h->flags[c] & FLAG_FIXED) ? 1 : 0;
        for (int k = 0; k < 3; ++k) f[k * n + c] = F[3 * c + k];
    }
    HIP_OK(h, hipMemcpyAsync(w + L.E, E.data(), n * 8, hipMemcpyHostToDevice, s));
    HIP_OK(h, hipMemcpyAsync(w + L.G, G.data(), n * 8, hipMemcpyHostToDevice, s));
    HIP_OK(h, hipMemcpyAsync(w + L.fixed, fixed.data(), n, hipMemcpyHostToDevice, s));
    HIP_OK(h, hipMemcpyAsync(w + L.f, f.data(), 6 * n * 8, hipMemcpyHostToDevice, s));
    StaticArgs a{};
    a.nx = h->nx; a.ny = h->ny; a.nz = h->nz; a.n = n;
    a.l = h->p.voxel_size;
    a.mat = (const uint8_t *)(h->ws + h->L.mat);
    a.fixed = (const uint8_t *)(w + L.fixed);
    a.E = (const double *)(w + L.E);
    a.G = (const double *)(w + L.G);
    double *x = (double *)(w + L.x), *r = (double *)(w + L.r), *z = (double *)(w + L.z);
    double *p = (double *)(w + L.p), *q = (double *)(w + L.q), *diag = (double *)(w + L.diag);
    double *part = (double *)(w + L.partials);
    const int nb = static_blocks(n);
    std::vector<double> hp(2 * (size_t)nb);
    // sums of the partials in workgroup order: one value per block (stride
    // 1) or two interleaved values (stride 2)
    auto sums = [&](int stride, double *a0, double *a1) -> int {
        HIP_OK(h, hipMemcpyAsync(hp.data(), part, (size_t)stride * nb * 8, hipMemcpyDeviceToHost, s));
        HIP_OK(h, hipStreamSynchronize(s));
        double s0 = 0.0, s1 = 0.0;
        for (int b = 0; b < nb; ++b) {
            s0 += hp[(size_t)stride * b];
            if (stride == 2) s1 += hp[2 * (size_t)b + 1];
        }
        *a0 = s0;
        if (a1) *a1 = s1;
        return VX_OK;
    };
    HIP_OK(h, launch_static_diag(a, diag, s));
    HIP_OK(h, launch_static_start(a, (const double *)(w + L.f), diag, x, r, z, p, part, s));
    double rz = 0.0, ff = 0.0;
    int rc = sums(2, &rz, &ff);
    if (rc) return rc;
    int it = 0;
    bool converged = ff == 0.0;
    const double fnorm = std::sqrt(ff);
    while (!converged && it < max_iter) {
        HIP_OK(h, launch_static_apply(a, p, q, part, s));
        double pq = 0.0;
        if ((rc = sums(1, &pq, nullptr))) return rc;
        if (!(pq > 0.0)) break;   // the operator is singular on p (a free body)
        const double alpha = rz / pq;
        HIP_OK(h, launch_static_step(a, alpha, p, q, diag, x, r, z, part, s));
        double rz_new = 0.0, rr = 0.0;
        if ((rc = sums(2, &rz_new, &rr))) return rc;
        ++it;
        if (std::sqrt(rr) <= rel_tol * fnorm) { converged = true; break; }
        HIP_OK(h, launch_static_dir(n, rz_new / rz, z, p, s));
        rz = rz_new;
    }
    // the true residual |f - K x| / |f| on the unknowns
    HIP_OK(h, launch_static_apply(a, x, q, part, s));
    std::vector<double> hx(6 * n), hq(6 * n);
    HIP_OK(h, hipMemcpyAsync(hx.data(), x, 6 * n * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipMemcpyAsync(hq.data(), q, 6 * n * 8, hipMemcpyDeviceToHost, s));
    HIP_OK(h, hipStreamSynchronize(s));
    double res = 0.0;
    for (long long c = 0; c < n; ++c) {
        if (!h->grid[c] || fixed[c]) continue;
        for (int k = 0; k < 6; ++k) {
            const double d = f[k * n + c] - hq[k * n + c];
            res += d * d;
        }
    }
    res = ff > 0.0 ? std::sqrt(res) / fnorm : 0.0;
    for (long long c = 0; c < n; ++c)
        for (int k = 0; k < 3; ++k) {
            if (u) u[3 * c + k] = hx[k * n + c];
            if (theta) theta[3 * c + k] = hx[(3 + k) * n + c];
        }
    if (iters) *iters = it;
    if (rel_residual) *rel_residual = res;
    if (!converged) return fail(h, VX_EUNSTABLE, "conjugate gradients did not reach rel_tol");
    return VX_OK;
}

}  // namespace
