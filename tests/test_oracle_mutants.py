"""Mutation tests of the oracle's pins: each case plants one plausible
mistake (a dropped term, a wrong sign, a wrong index, a transposed operand)
in a copy of the oracle source, builds it, and runs the fast pins against
it in a child process.  Some pin must fail for every mutant; the unmutated
copy, built the same way, must pass them all."""
import os
import subprocess
import sys

import pytest

from oracle import oracle as O

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "frelbm_oracle.c")
PINS = ["tests/test_oracle_node.py", "tests/test_oracle_stencils.py", "tests/test_oracle_brute.py",
        "tests/test_oracle_physics.py::test_p7_couette",
        "tests/test_oracle_physics.py::test_p4_conservation_moving_walls",
        "tests/test_oracle_consistent_init.py"]

# (name, text in the source, replacement, which occurrence)
MUTANTS = [
    ("feq quadratic term sign", "- CS2 * d);", "+ CS2 * d);", 0),
    ("geq quadratic term sign", "- CS2 * d);", "+ CS2 * d);", 1),
    ("Guo term without (c.u) c", "cu * c[i][a] / (CS2 * CS2)", "0.0 * cu", 0),
    ("g_0 complement sign", "out[0] = phi - rest;", "out[0] = phi + rest;", 0),
    ("kappa1 and kappa2 swapped in mu_phi", "out[1] = kappa1 / 8.0 * ps - kappa2 / 8.0 * pt +",
     "out[1] = kappa2 / 8.0 * ps - kappa1 / 8.0 * pt +", 0),
    ("Laplacian prefactor", "return 2.0 / CS2 * acc;", "return 3.0 / CS2 * acc;", 0),
    ("gradient components transposed", "g[a] += w[i] * c[i][a] * X[n];",
     "g[a] += w[i] * c[i][(a + 1) % 3] * X[n];", 0),
    ("force term sign", "F[a] = s->mur[x] * gr[a] + s->mup[x] * gp[a] - gpi[a];",
     "F[a] = s->mur[x] * gr[a] - s->mup[x] * gp[a] - gpi[a];", 0),
    ("velocity without the half force", "(s->jx[x] + 0.5 * F[0])", "(s->jx[x] + F[0])", 0),
    ("moving-wall bounce-back sign", "fs - 2.0 * w[i] * s->rho[x] * cu / CS2",
     "fs + 2.0 * w[i] * s->rho[x] * cu / CS2", 0),
    ("solid fill without lattice weights", "num += w[i] * X[n];", "num += X[n];", 0),
    ("pre-iterations without the Guo term", "- feq[i]) / tf + S[i];", "- feq[i]) / tf + 0.0 * S[i];", 1),
    ("g not reset after the pre-iterations", "or_geq(kind, ph0[x], s->mup[x], G, u, &s->g[x * q]);",
     "(void)G;", 0),
]


# mistakes in the ternary extension, against the ternary pins (the Laplace
# pin left out for time: brute force and the derivative pins decide)
PINS3 = ["tests/test_oracle_ternary.py", "-k", "not laplace"]
MUTANTS3 = [
    ("mu_psi without the binary potentials", "out[2] = m[2] - 0.5 * (m[0] + m[1]);", "out[2] = m[2];", 0),
    ("C2 with the wrong sign of psi", "0.5 * (rho - phi - psi)", "0.5 * (rho - phi + psi)", 0),
    ("force without the psi term", "+ s->muq[x] * gq[a] - gpi[a];", "- gpi[a];", 0),
    ("h relaxing with tau_g", "- heq[i]) / th;", "- heq[i]) / tg;", 0),
    ("h equilibrium with mu_phi", "or_geq(kind, s->psi[x], s->muq[x], G3, u, heq);",
     "or_geq(kind, s->psi[x], s->mup[x], G3, u, heq);", 0),
    ("h bounced with phi", "hs - 2.0 * w[i] * s->psi[x] * cu / CS2", "hs - 2.0 * w[i] * s->phi[x] * cu / CS2", 0),
    ("Laplacian of C2 with the wrong sign of psi", "0.5 * (lap_rho - lap_phi - lap_psi)",
     "0.5 * (lap_rho - lap_phi + lap_psi)", 0),
]


def _build(tmp_path, text):
    src = tmp_path / "oracle_copy.c"
    src.write_text(text)
    return O.compile_source(str(src), str(tmp_path / "oracle_copy.so"))


def _run_pins(lib, pins=PINS):
    env = dict(os.environ, FRELBM_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", *pins],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    return r.returncode, r.stdout[-2000:]


def test_unmutated_copy_passes_the_pins(tmp_path):
    code, out = _run_pins(_build(tmp_path, open(SRC).read()))
    assert code == 0, out


@pytest.mark.parametrize("name,old,new,occ", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_some_pin_catches_the_mutant(tmp_path, name, old, new, occ):
    text = open(SRC).read()
    parts = text.split(old)
    assert len(parts) > occ + 1, f"mutation site for '{name}' not found"
    mutated = old.join(parts[:occ + 1]) + new + old.join(parts[occ + 1:])
    assert mutated != text
    code, out = _run_pins(_build(tmp_path, mutated))
    assert code != 0, f"every pin passed with the mutant '{name}'"


def test_unmutated_copy_passes_the_ternary_pins(tmp_path):
    code, out = _run_pins(_build(tmp_path, open(SRC).read()), PINS3)
    assert code == 0, out


@pytest.mark.parametrize("name,old,new,occ", MUTANTS3, ids=[m[0] for m in MUTANTS3])
def test_some_ternary_pin_catches_the_mutant(tmp_path, name, old, new, occ):
    text = open(SRC).read()
    parts = text.split(old)
    assert len(parts) > occ + 1, f"mutation site for '{name}' not found"
    mutated = old.join(parts[:occ + 1]) + new + old.join(parts[occ + 1:])
    code, out = _run_pins(_build(tmp_path, mutated), PINS3)
    assert code != 0, f"every ternary pin passed with the mutant '{name}'"
