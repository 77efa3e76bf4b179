"""Planted mistakes in the oracle (on the CPU, in a scratch copy) must each fail at least one
pin that does not re-implement the oracle's own readings: the closed forms, invariants and
symmetries of the SGS stress and of the dynamic model (tests/test_oracle_sgs_stress.py,
tests/test_oracle_sgs.py without the plain-loop re-derivation, tests/test_oracle_duct.py).
Each entry: (what is planted, file, original text, planted text)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

MUTATIONS = [
    ("SGS term with the wrong sign in the explicit right-hand side", "oracle/substep.py",
     "return (-ax + sx + case.nu * lu, -ay + sy + case.nu * lv, -az + sz + case.nu * lw)",
     "return (-ax - sx + case.nu * lu, -ay - sy + case.nu * lv, -az - sz + case.nu * lw)"),
    ("SGS term with the wrong sign when every viscous term is implicit", "oracle/substep.py",
     "return (-ax + sx, -ay + sy, -az + sz)", "return (-ax - sx, -ay - sy, -az - sz)"),
    ("SGS stress divergence halved", "oracle/ops.py",
     "    return fx, fy, fz\n", "    return 0.5 * fx, 0.5 * fy, 0.5 * fz\n"),
    ("edge eddy viscosity taken at the cell instead of the four-centre mean", "oracle/ops.py",
     "nu12 = 0.25 * (nI + xp(nI) + yp(nI) + xp(yp(nI)))", "nu12 = nI"),
    ("alpha^2 of the 3-D and 2-D filters swapped", "oracle/sgs.py",
     "table = {3: 4.0, 2: 4.0 ** (2.0 / 3.0), 1: 2.0 ** (2.0 / 3.0)}",
     "table = {3: 4.0 ** (2.0 / 3.0), 2: 4.0, 1: 2.0 ** (2.0 / 3.0)}"),
    ("alpha^2 = 4 on every layer", "oracle/sgs.py",
     "table = {3: 4.0, 2: 4.0 ** (2.0 / 3.0), 1: 2.0 ** (2.0 / 3.0)}",
     "table = {3: 4.0, 2: 4.0, 1: 4.0}"),
    ("Simpson weights (1/6, 2/3, 1/6) in the x pass of the test filter", "oracle/sgs.py",
     "q = 0.25 * xm(q) + 0.5 * q + 0.25 * xp(q)", "q = xm(q) / 6.0 + 2.0 * q / 3.0 + xp(q) / 6.0"),
    ("Simpson weights in the z pass of the test filter", "oracle/sgs.py",
     "return 0.25 * qp[:-2] + 0.5 * qp[1:-1] + 0.25 * qp[2:]",
     "return qp[:-2] / 6.0 + 2.0 * qp[1:-1] / 3.0 + qp[2:] / 6.0"),
    ("M_ij without its factor 2", "oracle/sgs.py",
     "M.append(2.0 * delta2 * (F(smag * s[c]) - alpha2 * stmag * st[c]))",
     "M.append(delta2 * (F(smag * s[c]) - alpha2 * stmag * st[c]))"),
    ("L_ij with the wrong sign of its second term", "oracle/sgs.py",
     "L.append(F(vel[a] * vel[b]) - fvel[a] * fvel[b])", "L.append(F(vel[a] * vel[b]) + fvel[a] * fvel[b])"),
    ("off-diagonal terms of L:M and M:M counted once", "oracle/sgs.py",
     "wgt = 1.0 if a == b else 2.0          # symmetric", "wgt = 1.0 if a == b else 1.0          # symmetric"),
]

PINS = ["tests/test_oracle_sgs_stress.py", "tests/test_oracle_sgs.py", "tests/test_oracle_duct.py",
        "tests/test_oracle_substep.py"]


@pytest.mark.slow
@pytest.mark.parametrize("mutation", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_planted_mistake_is_caught(mutation, tmp_path):
    name, rel, old, new = mutation
    dst = tmp_path / "repo"
    for d in ("oracle", "synth", "tests"):
        shutil.copytree(os.path.join(ROOT, d), dst / d, ignore=shutil.ignore_patterns("__pycache__"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), dst / "pytest.ini")
    path = dst / rel
    src = path.read_text()
    assert src.count(old) == 1, f"mutation site not found: {old}"
    path.write_text(src.replace(old, new))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-m", "not gpu", "-k", "not plain_loops",
                        "-p", "no:cacheprovider"] + PINS, cwd=dst, capture_output=True, text=True, timeout=600)
    assert r.returncode == 1 and "failed" in r.stdout, f"{name} not caught:\n{r.stdout[-1500:]}"
