"""Planted mistakes in a copy of the CPU oracle must each fail at least one pin.

Every mutant is a one-line edit of dg_oracle.c that models a plausible
mistake (a dropped term, a wrong sign, index or operand, the other reading of
an ambiguous passage).  It is compiled to a temporary library on the CPU and
the pin suite is run against it in a subprocess; the mutant must be caught.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "dg_oracle.c")

MUTANTS = {
    "drop_interior_kappa_term": ("val += P->kappa * (avvx * jux + avvy * juy);", "val += 0.0;"),
    "drop_average_half": ("const double avux = 0.5 * eps * gxs[S][c]", "const double avux = eps * gxs[S][c]"),
    "upwind_on_outflow": ("if (!(bnK < 0.0)) continue;", "if (!(bnK > 0.0)) continue;"),
    "upwind_uses_inner_trace": ("val += bnK * (uout - uin) * vK;", "val += bnK * (uout + uin) * vK;"),
    "transposed_convection": ("if (useC) s += (b1 * gx[c] + b2 * gy[c]) * v[a];",
                              "if (useC) s += (b1 * gx[a] + b2 * gy[a]) * v[c];"),
    "interior_penalty_on_dirichlet": ("const double pen = P->sigma_D * eps / he;",
                                      "const double pen = P->sigma * eps / he;"),
    "literal_dirichlet_rhs_sign": ("double r = gd * (pen * v[a] + P->kappa * eps * dnv);",
                                   "double r = gd * (pen * v[a] - eps * dnv);"),
    "inflow_on_neumann_too": ("if (M->bnd_type[bi] == 1) { /* Neumann",
                              "if (0) { /* Neumann"),
    "inward_normal": ("const double nx = ey / len, ny = -ex / len; /* outward normal of K_i */",
                      "const double nx = -ey / len, ny = ex / len;"),
    "stroud_weight_quarter": ("w[m] = 0.125 * wa[i] * wb[j];", "w[m] = 0.25 * wa[i] * wb[j];"),
    "legendre_recurrence_sign": ("poly_axpy(-(double)p / (p + 1.0), &t2, &Q[p + 1]);",
                                 "poly_axpy((double)p / (p + 1.0), &t2, &Q[p + 1]);"),
    "jacobi_alpha_off_by_one": ("double al = 2.0 * p + 1.0;", "double al = 2.0 * p;"),
    "drop_neumann_data": ("for (int a = 0; a < n; ++a) rhs[K * n + a] += ds * gn * v[a];", "(void)gn;"),
    "volume_det_missing": ("const double dx = wv[g] * A.det;", "const double dx = wv[g];"),
    "reaction_derivative_drops_power": ("dr += p * c[p - 1] * up;", "dr += c[p - 1] * up;"),
    "reaction_det_missing": ("const double dx = w[g] * A.det;", "const double dx = w[g];"),
    "reaction_power_off_by_one": ("r += c[p - 1] * up;", "r += c[p - 1] * up * u;"),
    "monomial_exponents_swapped": ("B->phi[m].c[d - q][q] = 1.0;", "B->phi[m].c[q][d - q] = 1.0;"),
    "monomial_basis_ignored": ("if (basis == ORC_BASIS_MONOMIAL) {", "if (0) {"),
}


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_mutant_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, "mutation anchor not found exactly once: %r" % old
    mpath = tmp_path / "mutant.c"
    mpath.write_text(src.replace(old, new))
    so = tmp_path / "libmutant.so"
    subprocess.check_call(["gcc", "-O2", "-std=c11", "-D_DEFAULT_SOURCE", "-fPIC", "-shared", "-w",
                           str(mpath), "-o", str(so), "-lm"])
    env = dict(os.environ, DG_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        "-x", "-q", "-p", "no:cacheprovider", "-k", "not brute_force"],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, "mutant %s survived every pin:\n%s" % (name, r.stdout[-2000:])


# Planted mistakes in the oracle's Python part (its mesh refinement), run
# against a copy of the package placed first on the import path.
PY_MUTANTS = {
    "refine_inner_child_clockwise": ("tris += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, bc, ca]]",
                                     "tris += [[a, ab, ca], [ab, b, bc], [ca, bc, c], [ab, ca, bc]]", "refine"),
    "refine_midpoint_half_weight": ("new_nodes.append([0.5 * (nodes[a][0] + nodes[b][0]), 0.5 * (nodes[a][1] + nodes[b][1])])",
                                    "new_nodes.append([nodes[a][0] + 0.5 * nodes[b][0], 0.5 * (nodes[a][1] + nodes[b][1])])",
                                    "refine"),
    "refine_boundary_half_reversed": ("out += [[a, m], [m, b]]", "out += [[m, a], [m, b]]", "refine"),
    "euler_identity_mass": ("rhs = blocks.rhs + inv_dt * (M @ x)", "rhs = blocks.rhs + inv_dt * x", "euler"),
    "euler_one_step_short": ("    for _ in range(n_steps):\n        rhs = blocks.rhs", "    for _ in range(n_steps - 1):\n        rhs = blocks.rhs", "euler"),
    "newton_ignores_given_rhs": ("F = blocks.rhs if rhs is None else np.asarray(rhs, dtype=np.float64)",
                                 "F = blocks.rhs", "euler"),
}


@pytest.mark.parametrize("name", sorted(PY_MUTANTS) + ["unchanged_copy"])
def test_python_mutant_is_caught(name, tmp_path):
    """Each mutant fails a refinement pin; the unchanged copy passes them all
    (so a failure means the pins, not the harness)."""
    import shutil
    old, new, sel = PY_MUTANTS.get(name, ("def uniform_refine(", "def uniform_refine(", "refine or euler"))
    pkg = os.path.join(ROOT, "oracle")
    src = open(os.path.join(pkg, "__init__.py")).read()
    assert src.count(old) == 1, "mutation anchor not found exactly once: %r" % old
    dst = tmp_path / "oracle"
    dst.mkdir()
    for f in os.listdir(pkg):
        if f.endswith((".c", ".so", ".py")) and f != "__init__.py":
            shutil.copy(os.path.join(pkg, f), dst / f)
    (dst / "__init__.py").write_text(src.replace(old, new))
    # the mutant is imported first, so the pins (which pytest imports with the
    # repository at the front of the path) find it already loaded
    code = ("import sys; sys.path.insert(0, %r); import oracle; assert oracle.__file__.startswith(%r); "
            "sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main([%r, '-x', '-q', '-p', 'no:cacheprovider', '-k', %r]))"
            % (str(tmp_path), str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_oracle_pins.py"), sel))
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
    if name == "unchanged_copy":
        assert r.returncode == 0, r.stdout[-2000:]
    else:
        assert r.returncode != 0, "mutant %s survived every pin:\n%s" % (name, r.stdout[-2000:])


# Planted mistakes in the perceptron oracle (oracle/mlp.py): the pins of
# tests/test_mlp_oracle.py (hand-computed network, closed-form gradients,
# BF16 rounding, finite differences) must catch each.
MLP_MUTANTS = {
    "sigmoid_for_silu": ("return z / (1.0 + np.exp(-z))", "return 1.0 / (1.0 + np.exp(-z))"),
    "bias_dropped": ("z = H[-1] @ r(W).T + b", "z = H[-1] @ r(W).T"),
    "activation_on_last_layer": ("        if l < len(layers) - 1:\n            H.append(r(silu(z)))",
                                 "        H.append(r(silu(z)))\n        Z[-1] = silu(z)"),
    "silu_derivative_is_sigmoid_derivative": ("return s * (1.0 + z * (1.0 - s))", "return s * (1.0 - s)"),
    "bf16_truncates": ("u = (u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000", "u = u & 0xFFFF0000"),
    "weight_gradient_uses_next_activation": ("grads.append((r(dz).T @ H[l], dz.sum(axis=0)))",
                                             "grads.append((r(dz).T @ H[min(l + 1, len(H) - 1)], dz.sum(axis=0)))"),
}


@pytest.mark.parametrize("name", sorted(MLP_MUTANTS) + ["unchanged_copy"])
def test_mlp_mutant_is_caught(name, tmp_path):
    import shutil
    old, new = MLP_MUTANTS.get(name, ("import numpy as np", "import numpy as np"))
    pkg = os.path.join(ROOT, "oracle")
    src = open(os.path.join(pkg, "mlp.py")).read()
    assert src.count(old) == 1, "mutation anchor not found exactly once: %r" % old
    dst = tmp_path / "oracle"
    dst.mkdir()
    for f in os.listdir(pkg):
        if f.endswith((".c", ".so", ".py")) and f != "mlp.py":
            shutil.copy(os.path.join(pkg, f), dst / f)
    (dst / "mlp.py").write_text(src.replace(old, new))
    code = ("import sys; sys.path.insert(0, %r); import oracle.mlp; assert oracle.mlp.__file__.startswith(%r); "
            "sys.path.insert(1, %r); import pytest; "
            "sys.exit(pytest.main([%r, '-x', '-q', '-p', 'no:cacheprovider']))"
            % (str(tmp_path), str(tmp_path), ROOT, os.path.join(ROOT, "tests", "test_mlp_oracle.py")))
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True, text=True, timeout=600)
    assert "passed" in r.stdout or "failed" in r.stdout, r.stdout[-2000:] + r.stderr[-2000:]
    if name == "unchanged_copy":
        assert r.returncode == 0, r.stdout[-2000:]
    else:
        assert r.returncode != 0, "mutant %s survived every pin:\n%s" % (name, r.stdout[-2000:])
