"""The oracle's pins catch plausible mistakes: each case below plants one
mistake in a copy of the oracle (its C source or its Python wrapper), builds
the copy on the CPU and runs the pins of tests/test_oracle_pins.py against
it in a child process; the pins must fail for every planted mistake and pass
for the unchanged copy.  CPU only; the product is not involved."""
from __future__ import annotations

import os
import shutil
import subprocess
import sys
from concurrent.futures import ThreadPoolExecutor

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
ORACLE = os.path.join(ROOT, "oracle")
PINS = os.path.join(ROOT, "tests", "test_oracle_pins.py")

# (name, file, text in the oracle, planted replacement)
MUTATIONS = [
    ("stiffness weight W dropped", "c",
     "for (int i = 0; i < 3; i++) s2 += P->W[e] * Be[i * ne + a] * q[i];\n    Fe[a] = s2;",
     "for (int i = 0; i < 3; i++) s2 += Be[i * ne + a] * q[i];\n    Fe[a] = s2;"),
    ("off-diagonal of D transposed", "c",
     "D[1][2] = D[2][1] = Dk[4 * E + e] * s;\n  D[0][2] = D[2][0] = Dk[5 * E + e] * s;\n  const double *Be",
     "D[1][2] = D[2][1] = Dk[5 * E + e] * s;\n  D[0][2] = D[2][0] = Dk[4 * E + e] * s;\n  const double *Be"),
    ("tetrahedron B transposed", "c",
     "B[(e * 3 + i) * 4 + a] = C[1 + i][a];", "B[(e * 3 + i) * 4 + a] = C[a][1 + i];"),
    ("hexahedron volume from the centre point", "c",
     "        vol += det3(Jq);\n      }\n      V[e] = vol;",
     "        vol += det3(Jq);\n      }\n      V[e] = 8.0 * detJ0[e] + 0.0 * vol;"),
    ("lumped capacity without 1/n_e", "c",
     "C[k] += P->rho[e] * P->V[e] / ne * cfun(P, e, T[k], &dc);",
     "C[k] += P->rho[e] * P->V[e] * cfun(P, e, T[k], &dc);"),
    ("c(T) slope with the wrong sign", "c",
     "  *dc = P->c1[e];\n  return P->c0[e] + P->c1[e] * T;",
     "  *dc = -P->c1[e];\n  return P->c0[e] - P->c1[e] * T;"),
    ("convection sign flipped", "c",
     "double conv = -P->fh[f] * (T[k] - P->fTa[f]);",
     "double conv = P->fh[f] * (T[k] - P->fTa[f]);"),
    ("radiation without the ambient term", "c",
     "(pow(T[k] - P->Tz, 4) - pow(P->fTa[f] - P->Tz, 4));",
     "(pow(T[k] - P->Tz, 4));"),
    ("surface share not divided by the face's nodes", "c",
     "    double share = P->farea[f] / P->nfn;\n    for (int b = 0; b < P->nfn; b++) {\n      int32_t k",
     "    double share = P->farea[f];\n    for (int b = 0; b < P->nfn; b++) {\n      int32_t k"),
    ("update adds the conductive load", "c",
     "Tn[k] = T[k] + P->dt[k] * (Q[k] - F[k]) / C[k];",
     "Tn[k] = T[k] + P->dt[k] * (Q[k] + F[k]) / C[k];"),
    ("essential condition not re-applied", "c",
     "for (int64_t i = 0; i < P->ndir; i++) Tn[P->dir_nodes[i]] = P->dir_T[i];",
     "for (int64_t i = 0; i < 0; i++) Tn[P->dir_nodes[i]] = P->dir_T[i];"),
    ("k table read at the element mean temperature", "c",
     "  double s = 0;\n  for (int a = 0; a < P->ne; a++) {\n    double d;\n"
     "    s += kfac_node(P, e, Te[a], &d);\n    ds[a] = d / P->ne;\n  }\n  return s / P->ne;",
     "  double tb = 0, d;\n  for (int a = 0; a < P->ne; a++) tb += Te[a] / P->ne;\n"
     "  const double s = kfac_node(P, e, tb, &d);\n"
     "  for (int a = 0; a < P->ne; a++) ds[a] = d / P->ne;\n  return s;"),
    ("table interpolates from the wrong end of the segment", "c",
     "return f[i - 1] + (T - Tt[i - 1]) / h * (f[i] - f[i - 1]);",
     "return f[i] + (T - Tt[i - 1]) / h * (f[i] - f[i - 1]);"),
    ("quadrilateral area with misplaced Gauss points", "c",
     "sv[4] = {-1, -1, 1, 1};\n      const double g = 1.0 / sqrt(3.0);",
     "sv[4] = {-1, -1, 1, 1};\n      const double g = 0.5;"),
    ("hourglass stiffness without the volume", "c",
     "/ 3.0 * V[e] * bb;", "/ 3.0 * bb;"),
    ("adjoint drops the conductivity-slope term", "c",
     "out[kk[a]] -= Kmu[a] + dse[a] * muKT;", "out[kk[a]] -= Kmu[a];"),
    ("adjoint radiation slope 3 instead of 4", "c",
     "(P->fh[f] + 4.0 * P->sigma * P->feps[f] * d * d * d);",
     "(P->fh[f] + 3.0 * P->sigma * P->feps[f] * d * d * d);"),
    ("schedule ignores the starting step", "c",
     "Pn.pt_W = Wrows + ((step0 + n) % nrows) * P->npt;",
     "Pn.pt_W = Wrows + (n % nrows) * P->npt;"),
    ("critical step: radiation rate 3 sigma eps", "py",
     "coef = share * (self.fh + 4.0 * SIGMA_SB", "coef = share * (self.fh + 3.0 * SIGMA_SB"),
    ("critical step: whole face area per node", "py",
     "share = self.farea / self.nfn\n", "share = self.farea\n"),
    ("critical step: conductivity taken at T_lo only", "py",
     "smax = np.maximum(self.s0 + self.s1 * Tlo, self.s0 + self.s1 * Thi)",
     "smax = self.s0 + self.s1 * Tlo"),
    ("critical step: capacity taken at T_lo only", "py",
     "cmin = np.minimum(self.c0 + self.c1 * Tlo, self.c0 + self.c1 * Thi)",
     "cmin = self.c0 + self.c1 * Tlo"),
]


def _copy_oracle(dst, which=None, old=None, new=None):
    """A built copy of the oracle package under dst/oracle, with one planted
    mistake (every occurrence of `old` replaced by `new`), or none."""
    pkg = os.path.join(dst, "oracle")
    os.makedirs(pkg)
    for f in ("fedfem_oracle.c", "__init__.py", "build.py"):
        shutil.copy(os.path.join(ORACLE, f), pkg)
    if which is not None:
        path = os.path.join(pkg, "fedfem_oracle.c" if which == "c" else "__init__.py")
        src = open(path).read()
        assert src.count(old) >= 1, f"mutation anchor missing: {old!r}"
        open(path, "w").write(src.replace(old, new))
    subprocess.run(["gcc", "-O1", "-std=c11", "-fPIC", "-shared", "-fopenmp",
                    "-ffp-contract=off", "-fno-fast-math", os.path.join(pkg, "fedfem_oracle.c"),
                    "-o", os.path.join(pkg, "liboracle.so"), "-lm"], check=True)


def _pins(dst):
    env = dict(os.environ, FEDFEM_ORACLE_ROOT=dst, OMP_NUM_THREADS="1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    return r.returncode, r.stdout[-2000:]


def test_unchanged_copy_passes(tmp_path):
    _copy_oracle(str(tmp_path))
    rc, out = _pins(str(tmp_path))
    assert rc == 0, out


def test_every_planted_mistake_fails_a_pin(tmp_path):
    def run(i):
        name, which, old, new = MUTATIONS[i]
        d = str(tmp_path / f"m{i}")
        _copy_oracle(d, which, old, new)
        return name, _pins(d)

    with ThreadPoolExecutor(max_workers=4) as ex:
        results = list(ex.map(run, range(len(MUTATIONS))))
    survived = [name for name, (rc, _) in results if rc == 0]
    broken = [(name, out) for name, (rc, out) in results if rc not in (0, 1)]
    assert not broken, broken       # rc 1: pins ran and one failed
    assert not survived, f"no pin fails for: {survived}"
