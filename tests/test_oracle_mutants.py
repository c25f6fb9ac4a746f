"""The pins catch plausible mistakes in the oracle, planted on the CPU.

Each case copies oracle.c, plants one mistake in the copy, builds it and runs
the pins that must catch that mistake against the broken build, in a child
process: they must fail.  The unchanged copy, built the same way, must pass
the same pins, so a failure comes from the planted mistake and not from the
harness.  Nothing here touches the committed oracle or any GPU.
"""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE_C = os.path.join(ROOT, "oracle", "oracle.c")
PINS = "tests/test_oracle_pins.py"

_NESTEROV = [f"{PINS}::test_nesterov_gamma_sequence", f"{PINS}::test_nesterov_extrapolation_by_hand"]
_LOSS = [f"{PINS}::test_loss_closed_forms_in_pixels"]

# (name, text in oracle.c, replacement, pins that must catch it)
MUTANTS = [
    ("gamma index shifted by one: (s^(k+1) - 1) / s^(k+2) (eq. nesterov_scalar)",
     "        gam[a] = st->accelerate ? (s[a] - 1.0) / snext : 0.0;\n",
     "        double snext2 = (sqrt(4.0 * snext * snext + 1.0) + 1.0) / 2.0;\n"
     "        gam[a] = st->accelerate ? (snext - 1.0) / snext2 : 0.0;\n",
     _NESTEROV),
    ("sign of the momentum x - x^(k-1) flipped for camera centres (eq. nesterov_t)",
     "cbar[i].t[a] = st->c[i].t[a] + g * (st->c[i].t[a] - st->cm1[i].t[a]);",
     "cbar[i].t[a] = st->c[i].t[a] + g * (st->cm1[i].t[a] - st->c[i].t[a]);",
     _NESTEROV[1:]),
    ("sign of the momentum flipped for rotations before the projection (eq. nesterov_R)",
     "Mx[a] = st->c[i].R[a] + g * (st->c[i].R[a] - st->cm1[i].R[a]);",
     "Mx[a] = st->c[i].R[a] + g * (st->cm1[i].R[a] - st->c[i].R[a]);",
     _NESTEROV[1:]),
    ("sign of the momentum flipped for landmarks (eq. nesterov_l)",
     "lbar[3 * j + a] = st->l[3 * j + a] + g * (st->l[3 * j + a] - st->lm1[3 * j + a]);",
     "lbar[3 * j + a] = st->l[3 * j + a] + g * (st->lm1[3 * j + a] - st->l[3 * j + a]);",
     _NESTEROV[1:]),
    ("loss width left in pixels instead of delta / s internally (readings R7, R9)",
     "    double dl = st->delta / st->scale;\n",
     "    double dl = st->delta;\n",
     _LOSS),
    ("Huber branch above delta with the wrong constant (2 delta |e| - 2 delta^2)",
     "        return 2.0 * dl * sqrt(s) - dl * dl;\n",
     "        return 2.0 * dl * sqrt(s) - 2.0 * dl * dl;\n",
     _LOSS),
    ("Welsch exponent divided by delta instead of delta^2 (equal at delta = 1 in pixels only)",
     "        double ex = exp(-s / (dl * dl));\n",
     "        double ex = exp(-s / dl);\n",
     _LOSS),
]


def _build(tmp_path, name, text):
    from oracle.build import build_from
    src = tmp_path / f"{name}.c"
    src.write_text(text)
    return build_from(str(src), str(tmp_path / f"{name}.so"))


def _run_pins(lib, pins):
    env = dict(os.environ, DABA_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider", *pins],
                          cwd=ROOT, env=env, capture_output=True, text=True, timeout=300)


@pytest.fixture(scope="module")
def source():
    return open(ORACLE_C).read()


def test_unchanged_copy_passes_the_pins(tmp_path, source):
    lib = _build(tmp_path, "unchanged", source)
    r = _run_pins(lib, _NESTEROV + _LOSS)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]


@pytest.mark.parametrize("name,old,new,pins", MUTANTS, ids=[m[0].split(" (")[0] for m in MUTANTS])
def test_planted_mistake_is_caught(tmp_path, source, name, old, new, pins):
    assert source.count(old) == 1, f"the text to mutate is not unique in oracle.c: {old!r}"
    lib = _build(tmp_path, "mutant", source.replace(old, new))
    r = _run_pins(lib, pins)
    # 1 = tests ran and failed (not a collection or usage error)
    assert r.returncode == 1, f"{name}: pins passed or did not run\n" + r.stdout[-2000:] + r.stderr[-2000:]
