"""Planted mistakes in the oracle must fail at least one pin.

Each case rewrites one expression of oracle4.c (a coefficient, a sign, an
index, a dropped term, a transposed operand), builds the broken copy into a
temporary directory on the CPU and runs the pin tests against it in a
subprocess; the case passes when the pins fail.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle4.c")

MUTATIONS = {
    "d2_weight": ("static const double W2[5] = {-1.0, 16.0, -30.0, 16.0, -1.0};",
                  "static const double W2[5] = {-1.0, 16.0, -30.0, 15.0, -1.0};"),
    "d1_sign": ("static const double W1[5] = {1.0, -8.0, 0.0, 8.0, -1.0};",
                "static const double W1[5] = {-1.0, 8.0, 0.0, -8.0, 1.0};"),
    "lap_drop_z": ("return pt_d2(G, f, 0, dx[0], c) + pt_d2(G, f, 1, dx[1], c) + pt_d2(G, f, 2, dx[2], c);",
                   "return pt_d2(G, f, 0, dx[0], c) + pt_d2(G, f, 1, dx[1], c) + pt_d2(G, f, 1, dx[2], c);"),
    "fill_wrong_index": ("f[at(G, i, j, k)] = f[at(G, i, wrap(j, ny), k)];",
                         "f[at(G, i, j, k)] = f[at(G, i, wrap(j + 1, ny), k)];"),
    "mixed_transposed_A": ("s += A[3 * a + b] * d1[a] * d1[b];",
                           "s += A[3 * b + a] * d1[a] * d1[a];"),
    "mixed_drop_pair": ("for (b = a + 1; b < 3; b++)\n                        s += pt_dmix",
                        "for (b = a + 2; b < 3; b++)\n                        s += pt_dmix"),
    "rk4_weight": ("u[c] = u[c] + dt / 6.0 * (ku[0][c] + 2.0 * ku[1][c] + 2.0 * ku[2][c] + ku[3][c]);",
                   "u[c] = u[c] + dt / 6.0 * (ku[0][c] + 2.0 * ku[1][c] + 2.0 * ku[2][c] + 2.0 * ku[3][c]);"),
    "rk4_stage_dt": ("axpy_interior(&G, dt, u, ku[2], su);", "axpy_interior(&G, 0.5 * dt, u, ku[2], su);"),
    "adjoint_no_c2": ("w[c] = c2 ? c2[c] * lrho[c] : lrho[c];", "w[c] = lrho[c];"),
    "adjoint_stage_coeff": ("static const double astage[4] = {0.5, 0.5, 1.0, 0.0};",
                            "static const double astage[4] = {0.5, 1.0, 0.5, 0.0};"),
    "c2bar_wrong_stage": ("lus[c] = pt_lap(G, us[s], dx, c);", "lus[c] = pt_lap(G, us[0], dx, c);"),
}


@pytest.mark.parametrize("name", sorted(MUTATIONS))
def test_planted_mistake_is_caught(name, tmp_path):
    sys.path.insert(0, ROOT)
    from oracle import build as B
    old, new = MUTATIONS[name]
    src = open(SRC).read()
    assert src.count(old) == 1, f"mutation anchor for {name} not found exactly once"
    mpath = tmp_path / "oracle4_mut.c"
    mpath.write_text(src.replace(old, new))
    lib = B.build(src=str(mpath), lib=str(tmp_path / "liboracle4_mut.so"))
    env = dict(os.environ, ORACLE4_LIB=lib, OMP_NUM_THREADS="2")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutation {name} survived every pin:\n{r.stdout[-2000:]}"
