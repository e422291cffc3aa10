"""Mutation check of the oracle's pins.

Each mutant below plants one plausible mistake in a copy of the oracle (a dropped term,
a wrong sign, a transposed operand, a wrong index, a wrong comparison).  The pin suites
(test_oracle_pins.py, test_oracle_density.py) are then run against that copy in a
subprocess whose import path puts the mutated ``oracle`` package first; every mutant
must make at least one pin fail.  The mutants are chosen so that each part the pins
cover (projection, composite, partials, chain rule, sigma, pre-rendered accumulators,
loss, selection, Adam, densification) has at least one.
"""
import os
import shutil
import subprocess
import sys
import tempfile
from concurrent.futures import ThreadPoolExecutor


ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
C_SRC = "oit_oracle.c"
PY_SRC = "oracle.py"

# (name, file, [(old, new), ...]): every `old` must occur exactly once in the file
MUTANTS = [
    # projection (Sec. 3.1)
    ("dilation dropped", C_SRC, [("    p->cov[0] += ORC_DILATION;\n", "")]),
    ("conic off-diagonal sign", C_SRC, [("p->conic[1] = -p->cov[1] / det;", "p->conic[1] = p->cov[1] / det;")]),
    ("W transposed in T = J W", C_SRC, [("acc += p->J[3 * a + k] * W[3 * k + b];", "acc += p->J[3 * a + k] * W[3 * b + k];")]),
    ("rotation transposed", C_SRC, [("R[1] = 2.0 * (x * y - w * z);", "R[1] = 2.0 * (x * y + w * z);"),
                                    ("R[3] = 2.0 * (x * y + w * z);", "R[3] = 2.0 * (x * y - w * z);")]),
    ("cx for cy", C_SRC, [("p->mx = cam->fx * p->tc[0] / tz + cam->cx;", "p->mx = cam->fx * p->tc[0] / tz + cam->cy;")]),
    ("opacity sign", C_SRC, [("exp(-s->opacity_logit[i])", "exp(s->opacity_logit[i])")]),
    ("box extents swapped", C_SRC, [("hx = sqrt(p->tau * p->cov[0]), hy = sqrt(p->tau * p->cov[3]);",
                                     "hx = sqrt(p->tau * p->cov[3]), hy = sqrt(p->tau * p->cov[0]);")]),
    ("colour not clamped", C_SRC, [("p->color[ch] = p->raw_c[ch] > 0.0 ? p->raw_c[ch] : 0.0;",
                                    "p->color[ch] = p->raw_c[ch];")]),
    # weight and composite (Sec. 1, Sec. 3.2)
    ("v dropped from w", C_SRC, [("p->w = p->w_on ? (1.0 - p->d / sigma) * p->v : 0.0;",
                                  "p->w = p->w_on ? (1.0 - p->d / sigma) : 0.0;")]),
    ("1 - T dropped", C_SRC, [("C[ch] = a->T * bg[ch] + (1.0 - a->T) * F[ch];", "C[ch] = a->T * bg[ch] + F[ch];")]),
    ("alpha not capped", C_SRC, [("*capped = a > ORC_ALPHA_MAX;", "*capped = 0;")]),
    ("P1 without depth", C_SRC, [("a->P1[ch] += p->color[ch] * alpha * p->v * p->d;",
                                  "a->P1[ch] += p->color[ch] * alpha * p->v;")]),
    ("logT sign", C_SRC, [("a->logT += log(1.0 - alpha);", "a->logT += log(1.0 + alpha);")]),
    # partials (App. B) and the chain rule
    ("dC/dalpha without 1/(1 - alpha)", C_SRC, [("const double dC_dalpha = T / (1.0 - alpha) * (F - bg[ch]) +",
                                                 "const double dC_dalpha = T * (F - bg[ch]) +")]),
    ("dC/dw sign", C_SRC, [("const double dC_dw = Q > 0.0 ? (1.0 - T) * (alpha / Q) * (p->color[ch] - F) : 0.0;",
                            "const double dC_dw = Q > 0.0 ? (1.0 - T) * (alpha / Q) * (F - p->color[ch]) : 0.0;")]),
    ("dL/do by alpha", C_SRC, [("sg->opacity += dL_dalpha * G;", "sg->opacity += dL_dalpha * alpha;")]),
    # (sum_i w_i dL/dw_i = 0 makes v d / sigma^2 and v / sigma give the same total, so the
    # planted mistake is a power of sigma, not that equivalent form)
    ("sigma gradient power", C_SRC, [("*g_sigma += sg->w * p->v * p->d / (sigma * sigma);",
                                      "*g_sigma += sg->w * p->v * p->d / sigma;")]),
    ("dC/dw without c - F", C_SRC, [("const double dC_dw = Q > 0.0 ? (1.0 - T) * (alpha / Q) * (p->color[ch] - F) : 0.0;",
                                     "const double dC_dw = Q > 0.0 ? (1.0 - T) * (alpha / Q) * p->color[ch] : 0.0;")]),
    ("depth term of w dropped", C_SRC, [("        g_tc[2] += sg->w * (-p->v / sigma);\n", "")]),
    ("quaternion derivative entry", C_SRC, [("{2.0 * z, 2.0 * y, 2.0 * x, 2.0 * w},", "{2.0 * z, 2.0 * y, 2.0 * x, -2.0 * w},")]),
    ("guard-band derivative sign", C_SRC, [("g_tc[2] += g_J[2] * (cam->fx * (p->clamp_x * p->lim_x) / tz2);",
                                            "g_tc[2] += g_J[2] * (-cam->fx * (p->clamp_x * p->lim_x) / tz2);")]),
    ("direction normalisation dropped", C_SRC, [("g_mu[a] += (g_dir[a] - p->dir[a] * dd) / p->dist;",
                                                 "g_mu[a] += g_dir[a] / p->dist;")]),
    ("covariance chain index", C_SRC, [("acc += p->T[3 * k + a] * g_cov[2 * k + l] * p->T[3 * l + b];",
                                        "acc += p->T[3 * k + a] * g_cov[2 * k + l] * p->T[3 * l + a];")]),
    ("log-scale chain factor", C_SRC, [("gr->log_scale[(long)b * n + i] += gs * p->scale[b];",
                                        "gr->log_scale[(long)b * n + i] += gs;")]),
    # loss, activeness, selection, Adam (Sec. 4.1, Sec. 5.1)
    ("L1 gradient not divided", PY_SRC, [("return float(np.abs(d).sum() / n), np.sign(d) / n",
                                          "return float(np.abs(d).sum() / n), np.sign(d)")]),
    ("activeness for every group", PY_SRC, [("    s = np.zeros(len(rows))\n", "    s = np.full(len(rows), np.inf)\n"),
                                            ("s = np.maximum(s, nrm / eps[g])", "s = np.minimum(s, nrm / eps[g])")]),
    ("activeness L1 norm", PY_SRC, [("nrm = np.sqrt((np.asarray(grads[g], np.float64) ** 2).sum(axis=0))",
                                     "nrm = np.abs(np.asarray(grads[g], np.float64)).sum(axis=0)")]),
    ("threshold not strict", PY_SRC, [("np.nonzero(np.asarray(score) > thresh)", "np.nonzero(np.asarray(score) >= thresh)")]),
    ("top-k ties to the higher index", PY_SRC, [("key=lambda i: (-float(score[i]), i))", "key=lambda i: (-float(score[i]), -i))")]),
    ("label-change sign", PY_SRC, [("np.where(new_label[changed] == 1, -1, 1)", "np.where(new_label[changed] == 1, 1, -1)")]),
    ("Adam without bias correction", PY_SRC, [("mhat = m[:, rows] / (1.0 - beta1 ** step)", "mhat = m[:, rows]")]),
    # densification (Sec. 5.1, 3DGS's density control)
    ("clone and split swapped", PY_SRC, [("clone, split = cand & small, cand & ~small", "clone, split = cand & ~small, cand & small")]),
    ("statistic unit scaling", PY_SRC, [("math.hypot(scr[i, 0] * cam.width / 2.0, scr[i, 1] * cam.height / 2.0)",
                                         "math.hypot(scr[i, 0] * cam.width, scr[i, 1] * cam.height)")]),
    ("child offset rotated back", PY_SRC, [('child["mean"] = params["mean"][:, i] + R @ (s * np.asarray(z, np.float64))',
                                            'child["mean"] = params["mean"][:, i] + R.T @ (s * np.asarray(z, np.float64))')]),
    ("keep test non-strict", PY_SRC, [("& (np.asarray(uniform, f) < f(rules.keep_probability))",
                                       "& (np.asarray(uniform, f) <= f(rules.keep_probability))")]),
    ("opacity reset keeps moments", PY_SRC, [('    m["opacity_logit"] = np.zeros_like(m["opacity_logit"])\n', "")]),
]


def _make_copy(tmp, name, fname, subs):
    """A tree in tmp with the mutated oracle and links to the pins and the scene module."""
    ora = os.path.join(tmp, "oracle")
    os.makedirs(ora)
    for f in (C_SRC, PY_SRC):
        shutil.copy(os.path.join(ROOT, "oracle", f), os.path.join(ora, f))
    path = os.path.join(ora, fname)
    text = open(path).read()
    for old, new in subs:
        assert text.count(old) == 1, (name, old)
        text = text.replace(old, new)
    open(path, "w").write(text)
    os.symlink(os.path.join(ROOT, "tests"), os.path.join(tmp, "tests"))
    os.symlink(os.path.join(ROOT, "paper_2605_13855_amd"), os.path.join(tmp, "paper_2605_13855_amd"))
    shutil.copy(os.path.join(ROOT, "pytest.ini"), os.path.join(tmp, "pytest.ini"))


def _run_pins(tmp):
    env = dict(os.environ)
    env["PYTHONPATH"] = tmp
    env["PYTHONDONTWRITEBYTECODE"] = "1"
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
           "tests/test_oracle_pins.py", "tests/test_oracle_density.py"]
    r = subprocess.run(cmd, cwd=tmp, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def _one(m):
    name, fname, subs = m
    tmp = tempfile.mkdtemp(prefix="oracle_mutant_")
    try:
        _make_copy(tmp, name, fname, subs)
        return name, _run_pins(tmp)
    finally:
        shutil.rmtree(tmp, ignore_errors=True)


def test_every_mutant_fails_a_pin():
    """Each planted mistake makes the pins fail; the unmutated copy passes them (so that
    a failure comes from the mutation, not from the harness)."""
    rc, out = _one(("unmutated", PY_SRC, []))[1]
    assert rc == 0, out
    with ThreadPoolExecutor(max_workers=6) as ex:
        results = list(ex.map(_one, MUTANTS))
    survivors = [name for name, (rc, _) in results if rc == 0]
    assert not survivors, f"mutants that no pin catches: {survivors}"
    # a failing pin must be an assertion failure, not a crash of the harness
    for name, (rc, out) in results:
        assert rc == 1, (name, rc, out)
