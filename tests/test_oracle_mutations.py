"""Planted mistakes in the FP64 reference: each test compiles a copy of
oracle/wsr_oracle.c with one plausible error (a flipped sign, a dropped
term, a swapped operand or index, a wrong constant) and runs the reference's
own pins against it in a child process.  At least one pin must fail for
every mistake; a mistake that passes would mean the pins cannot tell a wrong
reference from a right one."""
import os
import subprocess
import sys

import pytest

import oracle

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "wsr_oracle.c")
PINS = ["tests/test_oracle_pins.py", "tests/test_oracle_grad.py", "tests/test_oracle_oit.py",
        "tests/test_oracle_sorted.py", "tests/test_oracle_earlyout.py"]

# (what the mistake is, text in the source, replacement); each text occurs in
# the source, and only its first occurrence is replaced
MUTATIONS = [
    ("rotation: sign of one quaternion term", "R[5] = 2.0 * (y * z - w * x);", "R[5] = 2.0 * (y * z + w * x);"),
    ("view transform: two coordinates swapped", "V[4 * r + 1] * p[1] + V[4 * r + 2] * p[2]",
     "V[4 * r + 1] * p[2] + V[4 * r + 2] * p[1]"),
    ("EWA Jacobian: sign of the off-diagonal term", "{cam->fx / tz, 0.0, -cam->fx * rx / tz,",
     "{cam->fx / tz, 0.0, cam->fx * rx / tz,"),
    ("Jacobian clamp: wrong limit", "const double limx = 1.3 * 0.5", "const double limx = 1.5 * 0.5"),
    ("dilation dropped on one axis", "o->cov[0] = cov[0] + P->dilation;", "o->cov[0] = cov[0];"),
    ("conic: sign of the off-diagonal", "o->conic[1] = -o->cov[1] / det;", "o->conic[1] = o->cov[1] / det;"),
    ("SH basis: an operand swapped", "Y[5] = 0.5 * sqrt(15.0 / pi) * y * z;", "Y[5] = 0.5 * sqrt(15.0 / pi) * x * z;"),
    ("SH colour: the +0.5 offset dropped", "o->raw[c] = acc + 0.5;", "o->raw[c] = acc;"),
    ("pixel centre: the +0.5 dropped", "const double dx = (double)px + 0.5 - g->mu[0];",
     "const double dx = (double)px - g->mu[0];"),
    ("Eq. 7 numerator: background weight dropped", "N3[c] = P->bg[c] * P->w_bg + num[3 * o + c];",
     "N3[c] = P->bg[c] + num[3 * o + c];"),
    ("backward: sign of dL/dq", "double dq = -0.5 * a * dLda;", "double dq = 0.5 * a * dLda;"),
]


@pytest.mark.parametrize("what,old,new", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_a_planted_mistake_fails_a_pin(tmp_path, what, old, new):
    text = open(SRC).read()
    assert old in text, what
    src = tmp_path / "wsr_oracle.c"
    src.write_text(text.replace(old, new, 1))
    lib = oracle.build(force=True, src=str(src), out=str(tmp_path / "liboracle.so"))
    env = dict(os.environ, WSR_ORACLE_LIB=lib)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                       + PINS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    # exit status 1: tests ran and one failed (not a collection or usage error)
    assert r.returncode == 1, (what, r.returncode, r.stdout[-2000:])
