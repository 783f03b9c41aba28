"""The pins have teeth: plausible mistakes planted in a copy of the oracle.

Each mutation below edits one spot of oracle/oracle.c (the kind of slip a
reader of the paper could make: a sign, an order, an index, a precision),
the altered copy is compiled into a library of its own, and the pin suite
(tests/test_oracle_pins.py) runs against it in a subprocess.  Every mutant
must fail at least one pin; the unaltered copy, built the same way, must pass
them all.  Runs on the CPU only.
"""
import os
import re
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

from oracle import build as orabuild

pytestmark = pytest.mark.slow

TESTS = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(TESTS)

# (name, text in oracle.c, replacement); the text must occur exactly once
MUTATIONS = [
    # the method (Sec. II-A to II-F, III-A)
    ("off-diagonal sign", "L->val[e] = (j == i) ? d : -1.0;", "L->val[e] = (j == i) ? d : 1.0;"),
    ("backward sweep in forward colour order",
     "for (int k = c - 1; k >= 0; --k) ora_colour_pass(h, level, k, r, z);",
     "for (int k = 0; k < c; ++k) ora_colour_pass(h, level, k, r, z);"),
    ("injection point off the octet corner",
     "F->f2c[j] = 2 * jx + (int64_t)F->nx * (2 * jy + (int64_t)F->ny * 2 * jz);",
     "F->f2c[j] = 2 * jx + 1 + (int64_t)F->nx * (2 * jy + (int64_t)F->ny * 2 * jz);"),
    ("beta inverted", "double beta = rho / rho_old;", "double beta = rho_old / rho;"),
    ("restriction sign", "rc[j] = r[i] - f[i];", "rc[j] = f[i] - r[i];"),
    ("greedy neighbour set misses the previous row", "if (j < i) used[L->colour[j]] = 1;",
     "if (j < i - 1) used[L->colour[j]] = 1;"),
    ("refinement weight",
     "const ora_level *C = &h->lev[level + 1];\n    for (int64_t j = 0; j < C->n; ++j) z[L->f2c[j]] += zc[j];",
     "const ora_level *C = &h->lev[level + 1];\n    for (int64_t j = 0; j < C->n; ++j) z[L->f2c[j]] += 0.5 * zc[j];"),
    ("gradient drops the logistic factor", "grad[i] = -lambda[i] * x[i] * logistic(theta[i]);",
     "grad[i] = -lambda[i] * x[i];"),
    ("residual update with p", "r[i] -= alpha * q[i];", "r[i] -= alpha * p[i];"),
    ("x update with q", "x[i] += alpha * p[i];", "x[i] += alpha * q[i];"),
    ("rho_old never updated", "        rho_old = rho;\n", "\n"),
    ("softplus without its linear part", "return (t > 0 ? t : 0.0) + log1p(exp(-fabs(t)));",
     "return log1p(exp(-fabs(t)));"),
    ("diagonal term not put back", "znew[t] = (r[i] - row_product(L, i, z) + z[i] * aii) / aii;",
     "znew[t] = (r[i] - row_product(L, i, z)) / aii;"),
    ("update in the off-diagonal form (other rounding)",
     "znew[t] = (r[i] - row_product(L, i, z) + z[i] * aii) / aii;",
     "znew[t] = (r[i] - (row_product(L, i, z) - z[i] * aii)) / aii;"),
    ("coarsest level smooths twice", "    smooth(h, level, r, z, lex);\n    if (level == h->levels - 1) return;",
     "    smooth(h, level, r, z, lex);\n    if (level == h->levels - 1) { smooth(h, level, r, z, lex); return; }"),
    # the sequential smoother (Sec. II-E, Eq. (1))
    ("sequential: sum over j < i only", "if (L->col[e] != i) acc += L->val[e] * z[L->col[e]];",
     "if (L->col[e] < i) acc += L->val[e] * z[L->col[e]];"),
    ("sequential: diagonal included in the sum", "if (L->col[e] != i) acc += L->val[e] * z[L->col[e]];",
     "acc += L->val[e] * z[L->col[e]];"),
    ("sequential: sign", "z[i] = (r[i] - acc) / L->diag[i];", "z[i] = (r[i] + acc) / L->diag[i];"),
    ("sequential: second forward sweep", "for (int64_t i = L->n - 1; i >= 0; --i) gs_row(L, i, r, z);",
     "for (int64_t i = 0; i < L->n; ++i) gs_row(L, i, r, z);"),
    ("sequential: no backward sweep", "for (int64_t i = L->n - 1; i >= 0; --i) gs_row(L, i, r, z);", ""),
    ("sequential: PCG falls back to the coloured V-cycle", "else if (precond == 3) ora_vcycle_lex(h, 0, r, z);",
     "else if (precond == 3) ora_vcycle(h, 0, r, z);"),
    ("sequential: coarse levels coloured", "vcycle_with(h, level + 1, rc, zc, lex);",
     "vcycle_with(h, level + 1, rc, zc, 0);"),
    # several sweeps per smoothing step
    ("sweeps on level 0 only", "for (int k = 0; k < h->sweeps; ++k) {\n        if (lex)",
     "for (int k = 0; k < (level == 0 ? h->sweeps : 1); ++k) {\n        if (lex)"),
    ("one post-smoothing sweep", "ora_prolong_add(h, level, zc, z);\n    smooth(h, level, r, z, lex);",
     "ora_prolong_add(h, level, zc, z);\n    if (lex) ora_sgs_lex(h, level, r, z); else ora_sgs(h, level, r, z);"),
    ("one pre-smoothing sweep",
     "memset(z, 0, (size_t)L->n * sizeof(double));\n    smooth(h, level, r, z, lex);",
     "memset(z, 0, (size_t)L->n * sizeof(double));\n    if (lex) ora_sgs_lex(h, level, r, z); else ora_sgs(h, level, r, z);"),
    ("FP32: one pre-smoothing sweep",
     "memset(z, 0, (size_t)L->n * sizeof(float));\n    for (int k = 0; k < h->sweeps; ++k) ora_sgs32(h, level, r, z);",
     "memset(z, 0, (size_t)L->n * sizeof(float));\n    ora_sgs32(h, level, r, z);"),
    ("FP32: one post-smoothing sweep",
     "z[L->f2c[j]] += zc[j];\n    for (int k = 0; k < h->sweeps; ++k) ora_sgs32(h, level, r, z);",
     "z[L->f2c[j]] += zc[j];\n    ora_sgs32(h, level, r, z);"),
    ("zero sweeps accepted", "if (sweeps < 1) return -1;", "if (sweeps < 0) return -1;"),
    # precision of the FP32 V-cycle and of the inner products
    ("FP32: sweep row sums accumulated in double",
     "    float acc = 0.0f;\n    for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) acc += L->val32[e]",
     "    double acc = 0.0;\n    for (int64_t e = L->rowptr[i]; e < L->rowptr[i + 1]; ++e) acc += (double)L->val32[e]"),
    ("FP32: residual for the restriction in double", "        float s = 0.0f;\n", "        double s = 0.0;\n"),
    ("FP32: update evaluated in double",
     "znew[t] = (r[i] - row_product32(L, i, z) + z[i] * aii) / aii;",
     "znew[t] = (float)(((double)r[i] - row_product32(L, i, z) + (double)z[i] * aii) / aii);"),
    ("FP32: FP64 diagonal", "float aii = L->diag32[i];", "double aii = L->diag[i];"),
    ("inner product as a plain double sum",
     "    long double s = 0.0L;\n    for (int64_t i = 0; i < n; ++i) s += (long double)a[i] * (long double)b[i];",
     "    double s = 0.0;\n    for (int64_t i = 0; i < n; ++i) s += a[i] * b[i];"),
]


def _run_pins(lib):
    env = dict(os.environ, MGPCG_ORACLE_LIB=lib, PYTHONDONTWRITEBYTECODE="1")
    cmd = [sys.executable, "-m", "pytest", os.path.join(TESTS, "test_oracle_pins.py"), "-x", "-q",
           "-p", "no:cacheprovider", "-o", "addopts="]
    r = subprocess.run(cmd, cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    failed = re.findall(r"FAILED \S+::(\S+)", r.stdout)
    return r.returncode, failed[0] if failed else r.stdout.strip().splitlines()[-1:]


def test_mutants_fail_a_pin(tmp_path):
    src = open(orabuild.SRC).read()
    jobs = [("unaltered", src)]
    for name, old, new in MUTATIONS:
        assert src.count(old) == 1, f"mutation '{name}': text occurs {src.count(old)} times"
        jobs.append((name, src.replace(old, new)))

    def one(k):
        name, text = jobs[k]
        c = tmp_path / f"m{k}.c"
        c.write_text(text)
        lib = str(tmp_path / f"libm{k}.so")
        orabuild.build_variant(str(c), lib)
        return name, *_run_pins(lib)

    with ThreadPoolExecutor(max_workers=min(8, os.cpu_count() or 1)) as ex:
        results = list(ex.map(one, range(len(jobs))))
    for name, rc, caught_by in results:
        print(f"{name:55s} rc={rc} {caught_by}")
    name, rc, info = results[0]
    assert rc == 0, f"the unaltered oracle fails its pins: {info}"
    survivors = [name for name, rc, _ in results[1:] if rc == 0]
    assert not survivors, f"mutants that pass every pin: {survivors}"
