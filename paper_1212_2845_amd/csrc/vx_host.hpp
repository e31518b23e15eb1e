// Host-side construction of the per-material and per-material-pair
// constants, shared by the single-lattice and batched front ends so that
// both feed the kernels identical numbers.
#pragma once

#include <algorithm>
#include <cmath>
#include <cstddef>
#include <new>
#include <vector>

#include "../../include/voxsim.h"
#include "vx_types.hpp"

namespace vx {

// Error code and message of an exception that reached a C entry point; the
// message is set only if that itself does not throw.
template <typename H>
int fail_nothrow(H *h, int code, const char *msg) noexcept {
    if (h) {
        try {
            h->err = msg;
        } catch (...) {
        }
    }
    return code;
}
inline int fail_nothrow(std::nullptr_t, int code, const char *) noexcept { return code; }

// Every C entry point runs its body between VX_TRY and VX_CATCH(handle), so
// that no C++ exception (host memory exhausted, say) crosses the interface.
#define VX_TRY try {
#define VX_CATCH(h)                                                                  \
    }                                                                                \
    catch (const std::bad_alloc &) {                                                 \
        return vx::fail_nothrow(h, VX_ENOMEM, "host memory exhausted");              \
    }                                                                                \
    catch (...) {                                                                    \
        return vx::fail_nothrow(h, VX_EDEVICE, "unexpected C++ exception");          \
    }

// Rest indices (x, y, z) of a voxel within its object packed as the
// collision kernels read them: 21 bits per axis, each offset by 2^20.
inline long long pack_ijk(int x, int y, int z) {
    const unsigned long long m = 0x1FFFFFull, b = 1ull << 20;
    return (long long)((((unsigned long long)(x + (int)b)) & m) | ((((unsigned long long)(y + (int)b)) & m) << 21) |
                       ((((unsigned long long)(z + (int)b)) & m) << 42));
}

// Composite of two moduli: springs of half length in series (Eq. 1, 2).
inline double composite(double a, double b) { return 2.0 * a * b / (a + b); }

// Voxel mass rho l^3 and inertia of a solid cube about its centre, m l^2/6.
inline double voxel_mass(const vx_material &M, double l) { return M.rho * l * l * l; }

template <typename T>
void build_tables(const vx_material *pal, int n_mat, const vx_params &p, std::vector<MatConst<T>> &mc,
                  std::vector<PairConst<T>> &pc) {
    const double l = p.voxel_size;
    mc.assign(n_mat, MatConst<T>{});
    for (int i = 1; i < n_mat; ++i) {
        const vx_material &M = pal[i];
        const double m = voxel_mass(M, l);
        const double I = m * l * l / 6.0;
        const double kv = M.E * l;              // voxel stiffness (floor, ground damping)
        const double kphi = M.E * l * l * l / 6.0;
        MatConst<T> &c = mc[i];
        c.m = (T)m; c.inv_m = (T)(1.0 / m); c.I = (T)I; c.inv_I = (T)(1.0 / I);
        c.cg = (T)(2.0 * p.zeta_slow * std::sqrt(m * kv));
        c.cgr = (T)(2.0 * p.zeta_slow * std::sqrt(I * kphi));
        c.cfloor = (T)(2.0 * p.zeta_col * std::sqrt(m * kv));
        c.kv = (T)kv; c.cte = (T)M.cte; c.mu_s = (T)M.mu_s; c.mu_d = (T)M.mu_d; c.E = (T)M.E;
        c.gfac = (T)(1.0 / (2.0 * (1.0 + M.nu)));
    }
    pc.assign((size_t)n_mat * n_mat, PairConst<T>{});
    for (int i = 1; i < n_mat; ++i)
        for (int j = 1; j < n_mat; ++j) {
            const vx_material &A = pal[i], &B = pal[j];
            const double Ec = composite(A.E, B.E);
            const double Gc = composite(A.E / (2.0 * (1.0 + A.nu)), B.E / (2.0 * (1.0 + B.nu)));
            // Eq. 8-12 with area l^2, I = l^4/12, J = l^4/6
            const double a1 = Ec * l;
            const double a2 = Gc * (l * l * l / 6.0);
            const double b3 = a1 * (l * l / 6.0);
            const double mmin = std::min(voxel_mass(A, l), voxel_mass(B, l));
            const double Imin = mmin * l * l / 6.0;
            PairConst<T> &c = pc[(size_t)i * n_mat + j];
            c.a1 = (T)a1; c.a2 = (T)a2; c.b1 = (T)a1; c.b2 = (T)(a1 * (0.5 * l)); c.b3 = (T)b3;
            c.ct = (T)(2.0 * p.zeta_bond * std::sqrt(mmin * a1));     // Eq. 34
            c.cr = (T)(2.0 * p.zeta_bond * std::sqrt(Imin * b3));     // Eq. 35
            c.kc = (T)a1;
            c.cc = (T)(2.0 * p.zeta_col * std::sqrt(mmin * a1));
        }
}

// Largest natural frequency sqrt(k_b / m_min) over the bonded material
// pairs marked in seen[n_mat * n_mat]; with no bond, over the voxels'
// own sqrt(E l / m) (marked in seen_vox[n_mat]).
inline double max_bond_omega(const vx_material *pal, int n_mat, double l, const std::vector<char> &seen,
                             const std::vector<char> &seen_vox) {
    double w = 0.0;
    bool any = false;
    for (int i = 1; i < n_mat; ++i)
        for (int j = 1; j < n_mat; ++j) {
            if (!seen[(size_t)i * n_mat + j]) continue;
            any = true;
            const double kb = composite(pal[i].E, pal[j].E) * l;
            const double mm = std::min(voxel_mass(pal[i], l), voxel_mass(pal[j], l));
            w = std::max(w, std::sqrt(kb / mm));
        }
    if (!any)
        for (int i = 1; i < n_mat; ++i)
            if (seen_vox[i]) w = std::max(w, std::sqrt(pal[i].E * l / voxel_mass(pal[i], l)));
    return w;
}

}  // namespace vx
