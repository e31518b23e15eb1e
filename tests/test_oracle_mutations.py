"""Mutation check of the oracle's pins (CPU only).

Each case plants one plausible mistake in a private copy of the oracle's C
source: a flipped sign, a transposed rotation, a wrong factor, a swapped axis,
a wrong composite rule, an extra integrator term, a wrong rest length, a
broken friction halt, a loosened lattice exclusion.  The copy is built in a
temporary directory and the pin suite runs against it in a subprocess (the
oracle package loads the build named by VX_ORACLE_LIB): some pin must fail.
A control copy without a change must pass a fast subset, so that a failure
is the planted mistake's and not the harness's.  The committed oracle is
never modified.
"""
import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")

MUTATIONS = {
    "z-force sign of the reduced end forces": ("b->b1 * Z2 + b->b2 * th.y", "b->b1 * Z2 - b->b2 * th.y"),
    "moment on voxel 1 applied with the stiffness sign":
        ("vec3 M1 = vscale(qrotate(A->q, perm_to_world(a, m1)), -1.0);",
         "vec3 M1 = vscale(qrotate(A->q, perm_to_world(a, m1)), 1.0);"),
    "separation taken into the bond frame by the transposed rotation":
        ("vec3 d = perm_to_local(a, qrotate_inv(A->q, dAB));", "vec3 d = perm_to_local(a, qrotate(A->q, dAB));"),
    "cross product of the damping's rigid spin reversed": ("vcross(r2, Wa)", "vcross(Wa, r2)"),
    "b3 factor of the moment on voxel 2": ("-b->b2 * Y2 + 2.0 * b->b3 * th.z", "-b->b2 * Y2 + b->b3 * th.z"),
    "rotational inertia of the voxel": ("V->I = V->m * l * l / 6.0;", "V->I = V->m * l * l / 12.0;"),
    "axis permutation of y-bonds": ("if (a == 1) return v3(v.y, v.z, v.x);", "if (a == 1) return v3(v.y, v.x, v.z);"),
    "composite modulus as the arithmetic mean": ("return 2.0 * a * b / (a + b);", "return 0.5 * (a + b);"),
    "extra term in the position update":
        ("V->U = vadd(V->U, vscale(vel, dt));",
         "V->U = vadd(V->U, vscale(vel, dt)); V->U = vadd(V->U, vscale(V->F, -dt * dt / V->m));"),
    "rest length from the summed, not the mean, strain":
        ("double L = l * (1.0 + 0.5 * (A->eps + B->eps));\n    /* Transform",
         "double L = l * (1.0 + (A->eps + B->eps));\n    /* Transform"),
    "friction halt test": ("if (vl <= V->mu_d * Fn * s->dt / V->m) {", "if (vl < 0.0) {"),
    "lattice exclusion of collision pairs": ("if (man <= 3) continue;", "if (man <= 2) continue;"),
    "contact separation reversed": ("vec3 r = separation(s, U, V);", "vec3 r = separation(s, V, U);"),
    "rotational bond damping with the larger inertia of the pair":
        ("double imin = A->I < B->I ? A->I : B->I;", "double imin = A->I > B->I ? A->I : B->I;"),
    "factor of the rotational bond damping":
        ("b->cr = 2.0 * s->p.zeta_bond * sqrt(imin * b->b3);", "b->cr = s->p.zeta_bond * sqrt(imin * b->b3);"),
    "rotational stiffness of the ground damping":
        ("V->kphi = mt->E * l * l * l / 6.0;", "V->kphi = mt->E * l * l * l / 12.0;"),
    "factor of the translational ground damping":
        ("F = vsub(F, vscale(vel, 2.0 * s->p.zeta_slow * sqrt(V->m * V->kv)));",
         "F = vsub(F, vscale(vel, s->p.zeta_slow * sqrt(V->m * V->kv)));"),
    "factor of 2 of the floor contact damping":
        ("double cd = 2.0 * s->p.zeta_col * sqrt(V->m * V->kv);", "double cd = s->p.zeta_col * sqrt(V->m * V->kv);"),
    "half of the floor spring energy": ("uf += 0.5 * V->kv * pen * pen;", "uf += V->kv * pen * pen;"),
    "gravitational energy at the rest height":
        ("ug += V->m * s->p.gravity * position(V).z;", "ug += V->m * s->p.gravity * V->D0.z;"),
    "rising slope of the triangle channel": ("if (x < 0.25) w = 4.0 * x;", "if (x < 0.25) w = 2.0 * x;"),
    "square channel switching a quarter period in": ("w = x < 0.5 ? 1.0 : -1.0;", "w = x < 0.25 ? 1.0 : -1.0;"),
    "channel offset dropped": ("return c->offset + c->amp * w;", "return c->amp * w;"),
    "channel frequency taken as an angular frequency":
        ("double theta = 2.0 * M_PI * c->freq * t + c->phase;", "double theta = c->freq * t + c->phase;"),
}


def _build(tmp, tag, change=None):
    d = os.path.join(str(tmp), tag)
    os.makedirs(d)
    src = open(os.path.join(ORACLE, "vx_oracle.c")).read()
    if change is not None:
        before, after = change
        assert src.count(before) == 1, tag
        src = src.replace(before, after)
    with open(os.path.join(d, "vx_oracle.c"), "w") as f:
        f.write(src)
    shutil.copy(os.path.join(ORACLE, "vx_oracle.h"), d)
    lib = os.path.join(d, "liboracle.so")
    subprocess.check_call(["gcc", "-std=c11", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fPIC", "-shared",
                           "-o", lib, os.path.join(d, "vx_oracle.c"), "-lm"])
    return lib


def _pins(lib, *extra):
    env = dict(os.environ, VX_ORACLE_LIB=lib)
    return subprocess.run([sys.executable, "-m", "pytest", os.path.join("tests", "test_oracle_pins.py"), "-x", "-q",
                           "-p", "no:cacheprovider"] + list(extra), cwd=ROOT, env=env, capture_output=True,
                          text=True)


def test_control_copy_passes_the_pins(tmp_path):
    lib = _build(tmp_path, "control")
    r = _pins(lib, "-k", "axial or timestep or free_fall or torsion or lazy_rebuild or static_friction")
    assert r.returncode == 0, r.stdout[-3000:]


def test_every_planted_mistake_fails_a_pin(tmp_path):
    libs = {name: _build(tmp_path, "m%02d" % i, change) for i, (name, change) in enumerate(MUTATIONS.items())}
    # the pins against the paper and the mathematics; the second
    # implementation of the step (the torch reference) is left out, so that
    # each mistake must fail a pin that does not compare with other code
    with ThreadPoolExecutor(4) as ex:
        codes = dict(zip(libs, ex.map(lambda name: _pins(libs[name], "-k", "not torch_reference").returncode, libs)))
    # exit code 1: a test failed; anything else would be the harness's fault
    assert all(rc == 1 for rc in codes.values()), codes
