"""Planted mistakes in the FP64 reference: each test builds a copy of the
renderer reference (oracle/wsr_oracle.c) or of the training reference
(oracle/train.py) with one plausible error (a flipped sign, a dropped term, a
swapped operand or index, a wrong constant) and runs the reference's own pins
against it in a child process.  At least one pin must fail for every
mistake; a mistake that passes would mean the pins cannot tell a wrong
reference from a right one."""
import concurrent.futures
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
    ("backward: factor 2 of the conic cross term dropped", "dcon[1] += dq * 2.0 * dx * dy;",
     "dcon[1] += dq * dx * dy;"),
    ("backward: mean gradient with dx and dy swapped",
     "dmu[1] += -dq * (2.0 * g->conic[1] * dx + 2.0 * g->conic[2] * dy);",
     "dmu[1] += -dq * (2.0 * g->conic[1] * dy + 2.0 * g->conic[2] * dx);"),
    ("backward: weight gradient through the wrong factor", "const double dw = das * g->u;",
     "const double dw = das * g->w;"),
    ("backward: sigmoid derivative term dropped", "g_logit[i] = du * g->u * (1.0 - g->u);",
     "g_logit[i] = du * g->u;"),
    ("backward: EXP beta gradient without its logarithm", "gbeta[j] = dw * (-P->sigma * db * log(d) * g->w);",
     "gbeta[j] = dw * (-P->sigma * db * g->w);"),
    ("OIT backward: 1 / (1 - alpha) dropped", "const double dLdal = -kfac[o] / (1.0 - al);",
     "const double dLdal = -kfac[o];"),
    ("early-out: cutoff without its factor 2", "const double c = 2.0 * log(o->u / P->alpha_cut);",
     "const double c = log(o->u / P->alpha_cut);"),
    ("sorted blending: transmittance not attenuated", "T *= 1.0 - a;", "T *= 1.0;"),
    ("OIT: coverage product without the clamp", "cov[o] *= 1.0 - clampd(g->u * G, 0.0, 1.0);",
     "cov[o] *= 1.0 - g->u * G;"),
    ("OIT: background and average weights swapped", "Cimg[3 * o + c] = cov[o] * P->bg[c] + (1.0 - cov[o]) * avg;",
     "Cimg[3 * o + c] = (1.0 - cov[o]) * P->bg[c] + cov[o] * avg;"),
    ("sorted blending: early stop ignored", "if (T < t_min) break;", "if (T < 0.0) break;"),
    ("box-restricted mode: red sum takes the green channel", "num[3 * o] += a * g->rgb[0];",
     "num[3 * o] += a * g->rgb[1];"),
    ("box-restricted mode: magnitude sum drops the absolute value", "aden[o] += fabs(a);", "aden[o] += a;"),
    ("ambiguity report: colour distance dropped", "sc += a * md;", "sc += a;"),
    ("ambiguity report: centre-rounding window a quarter too narrow",
     "return ldexp(gx * (fabs(dx) + pos_h) + gy * (fabs(dy) + pos_h), -24);",
     "return ldexp(gx * (fabs(dx) + pos_h) + gy * (fabs(dy) + pos_h), -26);"),
    ("early-out report: cutoff-rounding window a quarter as wide",
     "return 0x1p-23 * fabs(g->cut)", "return 0x1p-25 * fabs(g->cut)"),
    ("early-out report: cutoff-rounding window ten times as wide",
     "return 0x1p-23 * fabs(g->cut)", "return 10.0 * 0x1p-23 * fabs(g->cut)"),
    ("OIT strict mode: coverage without the clamp", "pc *= 1.0 - clampd(g->u * G, 0.0, 1.0);",
     "pc *= 1.0 - g->u * G;"),
    ("sorted blending: ambiguity report dropped",
     "if (fabs(q - tau) <= eta * M + amb_pos_window(g, dx, dy, pos_h)) amb += fabs(a);",
     "if (fabs(q - tau) <= eta * M + amb_pos_window(g, dx, dy, pos_h)) amb += 0.0;"),
    ("projection backward: factor 2 of d(T S T^T)/dT dropped", "dTm[c] = 2.0 * da * ST0[c] + dbv * ST1[c];",
     "dTm[c] = da * ST0[c] + dbv * ST1[c];"),
    ("projection backward: Sigma3D gradient not symmetrised",
     "acc += (dSig3[3 * r + k] + dSig3[3 * k + r]) * M[3 * k + l];", "acc += dSig3[3 * r + k] * M[3 * k + l];"),
    ("projection backward: exp of the log-scale not chained", "g_log_scales[l * n + i] = ds * s[l];",
     "g_log_scales[l * n + i] = ds;"),
    ("projection backward: quaternion normalisation not projected",
     "g_quats[k * n + i] = (dqh[k] - qh[k] * dot) / qn;", "g_quats[k * n + i] = dqh[k] / qn;"),
    ("projection backward: sign in the clamped Jacobian branch", "dt[2] += dJ[2] * (fx * rx / (tz * tz));",
     "dt[2] += dJ[2] * (-fx * rx / (tz * tz));"),
    ("projection backward: LC sigma gradient without the depth", "gsig[j] = dw * v_i * d / (P->sigma * P->sigma);",
     "gsig[j] = dw * v_i / (P->sigma * P->sigma);"),
    ("projection backward: view-direction normalisation not projected",
     "dp[c] = (ddir[c] - g->dir[c] * proj) / g->dist;", "dp[c] = ddir[c] / g->dist;"),
]


# an empty replacement: the unchanged copy, whose pins must all pass (shows that
# the failures below come from the planted mistakes, not from the set-up)
CONTROL = ("unchanged copy", "", "")

# the training reference (numpy): loss, its gradient and Adam
TRAIN_MUTATIONS = [
    ("SSIM: C1 not squared", "C1 = 0.01 ** 2", "C1 = 0.01"),
    ("SSIM: sign in the covariance term", "a2 = 2.0 * (sxy - u * v) + C2", "a2 = 2.0 * (sxy + u * v) + C2"),
    ("SSIM derivative: sign of dS/dSxx", "d_sxx = -s / b2", "d_sxx = s / b2"),
    ("loss gradient: x for y in the cross term", '+ y[..., ch] * filter2(t["d_sxy"], g)) / P',
     '+ x[..., ch] * filter2(t["d_sxy"], g)) / P'),
    ("l1 gradient: sign flipped", "grad = (1.0 - lam) * np.sign(x - y) / P", "grad = (1.0 - lam) * np.sign(y - x) / P"),
    ("Adam: first-moment bias correction dropped", "m_hat = m / (1.0 - beta1 ** step)", "m_hat = m"),
]


def _run_renderer_copy(tmp, old, new):
    """Build the C reference with `old` replaced by `new` and run its pins."""
    text = open(SRC).read()
    if old not in text:
        return None
    tmp.mkdir(parents=True)
    src = tmp / "wsr_oracle.c"
    src.write_text(text.replace(old, new, 1))
    lib = oracle.build(force=True, src=str(src), out=str(tmp / "liboracle.so"))
    env = dict(os.environ, WSR_ORACLE_LIB=lib, OMP_NUM_THREADS="2")
    return subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider", "-m", "not gpu"]
                          + PINS, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)


def _run_training_copy(tmp, old, new):
    """Import a copy of the training reference with `old` replaced by `new`
    ahead of the original and run its pins."""
    text = open(os.path.join(ROOT, "oracle", "train.py")).read()
    if old not in text:
        return None
    pkg = tmp / "oracle"
    pkg.mkdir(parents=True)
    (pkg / "train.py").write_text(text.replace(old, new, 1))
    (pkg / "__init__.py").write_text(open(os.path.join(ROOT, "oracle", "__init__.py")).read())
    env = dict(os.environ, WSR_ORACLE_LIB=oracle.build(force=False), OMP_NUM_THREADS="2")
    # the copy is imported first, so the pins' own import finds it
    code = (f"import sys; sys.path.insert(0, {str(tmp)!r}); import oracle.train; "
            f"assert oracle.train.__file__.startswith({str(tmp)!r}); import pytest; "
            "sys.exit(pytest.main(['-x', '-q', '-p', 'no:cacheprovider', 'tests/test_oracle_train.py']))")
    return subprocess.run([sys.executable, "-c", code], cwd=ROOT, env=env, capture_output=True, text=True,
                          timeout=600)


RENDERER_CASES = [CONTROL] + MUTATIONS
TRAINING_CASES = [CONTROL] + TRAIN_MUTATIONS


@pytest.fixture(scope="module")
def results(tmp_path_factory):
    """Every copy built and run once, four at a time; keyed by (reference, case)."""
    oracle.build(force=False)
    jobs = [("renderer", i, m) for i, m in enumerate(RENDERER_CASES)] + \
           [("training", i, m) for i, m in enumerate(TRAINING_CASES)]

    # the temporary directories are made here, in one thread (pytest's
    # temporary-directory factory is not safe to call from several threads)
    dirs = {(kind, i): tmp_path_factory.mktemp(f"{kind}{i}") for kind, i, _ in jobs}

    def run(job):
        kind, i, (_, old, new) = job
        fn = _run_renderer_copy if kind == "renderer" else _run_training_copy
        return (kind, i), fn(dirs[(kind, i)] / "copy", old, new)

    with concurrent.futures.ThreadPoolExecutor(max_workers=4) as pool:
        return dict(pool.map(run, jobs))


def _check(r, what, old):
    assert r is not None, f"{what}: the text to replace is not in the source"
    # exit status 1: tests ran and one failed (not a collection or usage error)
    assert r.returncode == (0 if not old else 1), (what, r.returncode, r.stdout[-2000:], r.stderr[-2000:])


@pytest.mark.parametrize("i", range(len(RENDERER_CASES)), ids=[m[0] for m in RENDERER_CASES])
def test_a_planted_mistake_fails_a_pin(results, i):
    what, old, _ = RENDERER_CASES[i]
    _check(results[("renderer", i)], what, old)


@pytest.mark.parametrize("i", range(len(TRAINING_CASES)), ids=[m[0] for m in TRAINING_CASES])
def test_a_planted_mistake_in_the_training_reference_fails_a_pin(results, i):
    what, old, _ = TRAINING_CASES[i]
    _check(results[("training", i)], what, old)
