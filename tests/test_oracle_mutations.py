"""Mutation check of the oracle's pins.

Each mutant is a copy of ``oracle/`` with one plausible mistake planted in its
arithmetic (a dropped factor, a wrong sign or index, a swapped operand, a wrong
averaging weight ...).  The pins of ``test_oracle_trajectory.py`` and
``test_oracle_pins.py`` run against every mutant in a subprocess; the check passes
when every mutant fails at least one pin and the unmutated copy, run through the same
harness, passes (the full pin set runs unmutated in the suite itself).
The mutants live in a temporary directory: nothing under ``oracle/`` is modified.

    python tests/test_oracle_mutations.py     # prints one line per mutant
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PIN_FILES = ["test_oracle_trajectory.py", "test_oracle_pins.py"]

C, PY = "oracle.c", "__init__.py"
# (name, file, text, replacement[, pin selection]); each text occurs exactly once in its
# file.  A selection (a pytest -k expression) narrows the pins run against that mutant to
# those that read the mutated code, which keeps the whole check short.
MUTANTS = [
    ("averaging 0.4 old + 0.6 tilde (f)", C, "f[i] = 0.5 * (f[i] + ft[i]);",
     "f[i] = 0.4 * f[i] + 0.6 * ft[i];"),
    ("averaging 0.4 old + 0.6 tilde (g)", C, "g[j] = 0.5 * (g[j] + gt[j]);",
     "g[j] = 0.4 * g[j] + 0.6 * gt[j];"),
    ("averaging 0.4 old + 0.6 tilde (p)", C, "p[i] = 0.5 * (p[i] + pt[i]);",
     "p[i] = 0.4 * p[i] + 0.6 * pt[i];"),
    ("averaging 0.4 old + 0.6 tilde (q)", C, "q[j] = 0.5 * (q[j] + qt[j]);",
     "q[j] = 0.4 * q[j] + 0.6 * qt[j];"),
    ("no averaging (f)", C, "f[i] = 0.5 * (f[i] + ft[i]);", "f[i] = ft[i];"),
    ("Gauss-Seidel: g~ from the new f~", C,
     "oracle_softmin_p(m, n, d, y, x, a, f, eps, lam, pexp, gt); /* a~^{alpha->beta}_j  */\n"
     "        oracle_softmin_p(n, m, d, x, y, b, g, eps, lam, pexp, ft);",
     "oracle_softmin_p(n, m, d, x, y, b, g, eps, lam, pexp, ft);\n"
     "        oracle_softmin_p(m, n, d, y, x, a, ft, eps, lam, pexp, gt);"),
    ("wrong potential in the alpha->beta softmin", C,
     "oracle_softmin_p(m, n, d, y, x, a, f, eps, lam, pexp, gt);",
     "oracle_softmin_p(m, n, d, y, x, a, p, eps, lam, pexp, gt);"),
    ("dropped 1/2 of the quadratic cost", C, "return pexp == 2.0 ? 0.5 * s :",
     "return pexp == 2.0 ? s :"),
    ("dropped 1/p of the cost", C, "pow(s, 0.5 * pexp) / pexp;", "pow(s, 0.5 * pexp);",
     "cost_p"),
    ("wrong power of the cost", C, "pow(s, 0.5 * pexp) / pexp;", "pow(s, pexp) / pexp;",
     "cost_p"),
    ("eps = sigma^2 for every p", C, "eps = power_p(sigma, pexp);", "eps = sigma * sigma;",
     "cost_p"),
    ("lambda with (sigma/reach)^2 for every p", C, "return 1.0 / (1.0 + power_p(t, pexp));",
     "return 1.0 / (1.0 + t * t);", "cost_p"),
    ("lambda without its exponent", C, "return 1.0 / (1.0 + power_p(t, pexp));",
     "return 1.0 / (1.0 + t);"),
    ("dropped lambda in the softmin", C, "out[i] = -lam * eps * (mx + log(sum));",
     "out[i] = -eps * (mx + log(sum));"),
    ("dropped log-weight", C, "s[j] = log(w[j]) + (h[j] - cost_p(", "s[j] = (h[j] - cost_p("),
    ("sign of the potential in the softmin", C, "(h[j] - cost_p(r + i * d", "(-h[j] - cost_p(r + i * d"),
    ("schedule starts one step low", C, "sigmas[k] = diameter * pow(scaling, (double)k);",
     "sigmas[k] = diameter * pow(scaling, (double)(k + 1));"),
    ("schedule one value short", C, "int K = (int)ceil(log(diameter / blur) / log(1.0 / scaling));",
     "int K = (int)floor(log(diameter / blur) / log(1.0 / scaling));"),
    ("bounding box ignores y's maximum", C, "if (y[j * d + k] > hi) hi = y[j * d + k];", ";"),
    ("eq. (6) coefficient rho + eps", C, "return -(rho + 0.5 * eps) * s;", "return -(rho + eps) * s;"),
    ("eq. (6) balanced: sign of the beta term", C, "s += b[j] * (g[j] - q[j]);",
     "s += b[j] * (q[j] - g[j]);"),
    ("eq. (6) unbalanced: reference e^{-f/rho}", C,
     "s += a[i] * exp(-p[i] / rho) * expm1(-(f[i] - p[i]) / rho);",
     "s += a[i] * exp(-f[i] / rho) * expm1(-(f[i] - p[i]) / rho);"),
    ("eq. (3) entropic term without eps", C, "return s1 + s2 + eps * s3;", "return s1 + s2 + s3;"),
    ("eq. (3) unbalanced: sign inside expm1", C, "rho * a[i] * (-expm1(-f[i] / rho))",
     "rho * a[i] * (-expm1(f[i] / rho))"),
    ("eq. (2) one marginal penalty dropped", C, "s += rho * (k1 + k2);", "s += rho * k1;"),
    ("marginal error without lambda", C, "exp((f[i] - ft[i] / lam) / eps)",
     "exp((f[i] - ft[i]) / eps)"),
    ("marginal error: balanced target when unbalanced", C,
     "a[i] : a[i] * exp(-f[i] / power_p(reach, pexp));", "a[i] : a[i];"),
    ("plan apply: eq. (7) flag inverted", C, "if (!divide_by_a) k *= a[i];",
     "if (divide_by_a) k *= a[i];"),
    ("gradient: sign of the cross term", C, "grad[i * d + k] += pij * (x[i * d + k] - y[j * d + k]);",
     "grad[i * d + k] -= pij * (x[i * d + k] - y[j * d + k]);"),
    ("gradient: sign of the self term", C, "grad[i * d + k] -= pil * (x[i * d + k] - x[l * d + k]);",
     "grad[i * d + k] += pil * (x[i * d + k] - x[l * d + k]);"),
    ("gradient: self plan without a_l", C, "double pil = a[i] * a[l] * exp(",
     "double pil = a[i] * exp("),
    ("weight gradient factor rho + eps/2", C, "out[i] = -(rho + eps) * exp(-p[i] / rho)",
     "out[i] = -(rho + 0.5 * eps) * exp(-p[i] / rho)"),
    ("weight gradient sign, balanced", C, "out[i] = f[i] - p[i];", "out[i] = p[i] - f[i];"),
    ("flips reverse coordinates instead of points", PY, "[:, ::-1, :]", "[:, :, ::-1]"),
    ("flipped half of the subject dropped", PY, "lab = lab[:n] + lab[n:]", "lab = lab[:n]",
     "label_transfer"),
    ("flipped copies at half weight", PY, "as_ = np.concatenate([a, a])",
     "as_ = np.concatenate([a, 0.5 * a])", "label_transfer"),
    ("grad_y with the potentials swapped", PY, "return grad_x(y, b, x, a, g, f, q, eps)",
     "return grad_x(y, b, x, a, f, g, q, eps)"),
    ("eq. (5) mass term sign", PY, "+ 0.5 * eps * (ma - mb) ** 2", "- 0.5 * eps * (ma - mb) ** 2"),
    ("barycenter: step without lr", PY, "x = x - lr * (grad / len(maps)) / a[:, None]",
     "x = x - (grad / len(maps)) / a[:, None]"),
    ("barycenter: sum over maps instead of mean", PY,
     "x = x - lr * (grad / len(maps)) / a[:, None]", "x = x - lr * grad / a[:, None]"),
    ("barycenter: no division by the support weight", PY,
     "x = x - lr * (grad / len(maps)) / a[:, None]", "x = x - lr * (grad / len(maps))"),
    ("barycenter: history sums the maps' S", PY, "hist.append(tot / len(maps))",
     "hist.append(tot)"),
]


def _run(mutant, workdir: str, threads: int = 2, select: str = ""):
    """Copies oracle/ (mutated when mutant is given) and the pin files into workdir
    and runs the pins there (those matching the mutant's selection, or `select`);
    returns (name, pytest return code, last output line)."""
    name = mutant[0] if mutant else "unmutated"
    if mutant and len(mutant) > 4:
        select = mutant[4]
    os.makedirs(os.path.join(workdir, "tests"))
    shutil.copytree(os.path.join(ROOT, "oracle"), os.path.join(workdir, "oracle"),
                    ignore=shutil.ignore_patterns("*.so", "*.tmp", "__pycache__"))
    os.symlink(os.path.join(ROOT, "synth"), os.path.join(workdir, "synth"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), workdir)
    for f in ["conftest.py"] + PIN_FILES:
        shutil.copy(os.path.join(ROOT, "tests", f), os.path.join(workdir, "tests", f))
    if mutant:
        fname, old, new = mutant[1:4]
        path = os.path.join(workdir, "oracle", fname)
        src = open(path).read()
        if src.count(old) != 1:
            return name, -1, f"mutation text found {src.count(old)} times"
        open(path, "w").write(src.replace(old, new))
    env = dict(os.environ, OMP_NUM_THREADS=str(threads), PYTHONDONTWRITEBYTECODE="1")
    env.pop("PYTHONPATH", None)
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *(["-k", select] if select else []),
                        *[os.path.join("tests", f) for f in PIN_FILES]],
                       cwd=workdir, env=env, capture_output=True, text=True, timeout=600)
    lines = [ln for ln in r.stdout.splitlines() if ln.strip()]
    return name, r.returncode, lines[-1] if lines else r.stderr[-200:]


def run_all(workers: int = 4, base_select: str = "trajectory or dirac"):
    """Results of the unmutated copy (on the pins matching base_select: the full set
    runs in the test suite itself) followed by every mutant."""
    base = tempfile.mkdtemp(prefix="oracle_mut_")
    try:
        jobs = [None] + MUTANTS
        with ThreadPoolExecutor(max_workers=workers) as ex:
            futs = [ex.submit(_run, m, os.path.join(base, f"m{k:02d}"), 2,
                              "" if m else base_select) for k, m in enumerate(jobs)]
            return [f.result() for f in futs]
    finally:
        shutil.rmtree(base, ignore_errors=True)


def test_every_mutant_fails_a_pin():
    res = run_all()
    name, rc, last = res[0]
    assert rc == 0, f"the unmutated oracle must pass its pins: {last}"
    survivors = [(n, rc, last) for n, rc, last in res[1:] if rc != 1]
    assert not survivors, f"mutants not caught (or broken harness): {survivors}"


if __name__ == "__main__":
    for name, rc, last in run_all():
        status = "passes" if name == "unmutated" and rc == 0 else ("caught" if rc == 1 else f"rc={rc}")
        print(f"{status:8s} {name:55s} {last}")
