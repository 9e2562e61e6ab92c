"""The oracle's pins must be able to fail: plant one plausible mistake at a
time in a copy of the oracle (on the CPU), rebuild it, and check that the pin
suite rejects every copy."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "omt_oracle.c")

MUTANTS = [
    ("wrong neighbour in div_x", "double yl = (j > 0) ? uy[I3(i, j - 1, c, n, k)]", "double yl = (j > 1) ? uy[I3(i, j - 2 + 1, c, n, k)]"),
    ("dropped extrapolation", "W->bx[q] = 2.0 * ux1[q] - ux[q];", "W->bx[q] = ux1[q];"),
    ("wrong u threshold", "orc_shrink_u(p->unorm, k, bx, by, p->mu);", "orc_shrink_u(p->unorm, k, bx, by, 0.9 * p->mu);"),
    ("sign of div_G", "x[c] = -s;", "x[c] = s;"),
    ("1/mu on the w block of R", "out[0] = su / p->mu + (l > 0 ? sw / p->nu", "out[0] = su / p->mu + (l > 0 ? sw / p->mu"),
    ("dropped source term", "phi1[q] = phi[q] + p->tau * (W->dx[q] + W->dg[q] + f[q]);", "phi1[q] = phi[q] + p->tau * (W->dx[q] + W->dg[q]);"),
    ("transposed gradient", "gy[I3(i, j, c, n, k)] = (j < n - 1) ? (phi[I3(i, j + 1, c, n, k)]", "gy[I3(i, j, c, n, k)] = (j < n - 1) ? (phi[I3(i + 1 < m ? i + 1 : i, j, c, n, k)]"),
    ("w threshold without alpha", "orc_shrink_w(p->wnorm, l, b, p->alpha * p->nu);", "orc_shrink_w(p->wnorm, l, b, p->nu);"),
    ("mu rule of S-OMT used for V-OMT", "p->mu = p->h * p->h / (32.0 * p->tau);", "p->mu = p->h * p->h / (16.0 * p->tau);"),
    ("regularised w factor with mu", "for (int e = 0; e < l; ++e) b[e] /= 1.0 + 2.0 * p->nu * p->eps;",
     "for (int e = 0; e < l; ++e) b[e] /= 1.0 + 2.0 * p->mu * p->eps;"),
    ("regularised w factor dropped", "for (int e = 0; e < l; ++e) b[e] /= 1.0 + 2.0 * p->nu * p->eps;",
     "for (int e = 0; e < l; ++e) b[e] /= 1.0;"),
    ("w dropped from the regulariser's objective", "for (size_t q = 0; q < Pl; ++q) sq += w1[q] * w1[q];",
     "for (size_t q = 0; q < Pl; ++q) sq += 0.0 * w1[q];"),
    ("sign of div_G in the constraint residual", "double r = t1[q] + (l > 0 ? t2[q] : 0.0) + f[q];",
     "double r = t1[q] - (l > 0 ? t2[q] : 0.0) + f[q];"),
    ("div_x dropped from the constraint residual", "double r = t1[q] + (l > 0 ? t2[q] : 0.0) + f[q];",
     "double r = (l > 0 ? t2[q] : 0.0) + f[q];"),
    ("constraint residual not relative to ||f||", "info->mass_residual = ff > 0 ? sqrt(met[3] / ff) : 0.0;",
     "info->mass_residual = ff > 0 ? sqrt(met[3]) : 0.0;"),
    ("gap relative to the dual", "info->rel_gap = met[1] > 0 ? (met[1] - met[2]) / met[1] : 0.0;",
     "info->rel_gap = met[1] > 0 ? (met[1] - met[2]) / met[2] : 0.0;"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,old,new", MUTANTS, ids=[m[0] for m in MUTANTS])
def test_pins_reject_mutant(tmp_path, name, old, new):
    src = open(SRC).read()
    assert old in src, f"pattern for '{name}' not found"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), str(mut), "-lm"],
                   check=True)
    env = dict(os.environ, OMT_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_operators.py"),
                        os.path.join(ROOT, "tests", "test_oracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant '{name}' survived the pins:\n{r.stdout[-2000:]}"


MSRC = os.path.join(ROOT, "oracle", "momt_oracle.c")

MATRIX_MUTANTS = [
    ("commutator order in grad_L", "Z[s * k * k + q] = LX[q] - XL[q];", "Z[s * k * k + q] = XL[q] - LX[q];"),
    ("missing conjugate in the inner product", "s += creal(X[q] * conj(Y[q]));", "s += creal(X[q] * Y[q]);"),
    ("dropped W extrapolation", "Wk->bw[q] = 2.0 * w1[q] - w[q];", "Wk->bw[q] = w1[q];"),
    ("nuclear shrink loses the sign", "g[p] = r > 0.0 ? (ev[p] > 0.0 ? r : -r) : 0.0;", "g[p] = r > 0.0 ? r : 0.0;"),
    ("skew shrink mapped back with +i", "for (int q = 0; q < kk; ++q) Xs[q] = -I * G[q];",
     "for (int q = 0; q < kk; ++q) Xs[q] = I * G[q];"),
    ("nu without the factor 4", "p->nu = lm > 0.0 ? 1.0 / (4.0 * p->tau * lm) : 0.0;",
     "p->nu = lm > 0.0 ? 1.0 / (2.0 * p->tau * lm) : 0.0;"),
    ("trace mean kept in f", "for (int a = 0; a < k; ++a) f[q * kk + a * k + a] -= mean;",
     "for (int a = 0; a < k; ++a) f[q * kk + a * k + a] -= 0.0 * mean;"),
    ("sign in the real image of a Hermitian matrix", "S[a * n + (k + b)] = -B;", "S[a * n + (k + b)] = B;"),
    ("mu rule of S-OMT", "if (p->mu <= 0.0) p->mu = p->h * p->h / (32.0 * p->tau);",
     "if (p->mu <= 0.0) p->mu = p->h * p->h / (16.0 * p->tau);"),
    ("W threshold without alpha", "morc_shrink_block(p->wnorm, 0, k, l, (double *)b, p->alpha * p->nu);",
     "morc_shrink_block(p->wnorm, 0, k, l, (double *)b, p->nu);"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,old,new", MATRIX_MUTANTS, ids=[m[0] for m in MATRIX_MUTANTS])
def test_matrix_pins_reject_mutant(tmp_path, name, old, new):
    src = open(MSRC).read()
    assert old in src, f"pattern for '{name}' not found"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), SRC, str(mut),
                    "-lm"], check=True)
    env = dict(os.environ, OMT_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_moracle_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant '{name}' survived the pins:\n{r.stdout[-2000:]}"


SRC3 = os.path.join(ROOT, "oracle", "omt3_oracle.c")

GRID3_MUTANTS = [
    ("u_z left out of the flux block", "double v[3] = {bx[c], by[c], bz[c]};", "double v[3] = {bx[c], by[c], 0.0};"),
    ("wrong z neighbour in div_x", "zl = z > 0 ? uz[ID4(i, j, z - 1, c, n, p, k)] : 0.0;",
     "zl = z > 1 ? uz[ID4(i, j, z - 2, c, n, p, k)] : 0.0;"),
    ("z gradient towards z - 1", "gz[o] = z < p - 1 ? (phi[ID4(i, j, z + 1, c, n, p, k)] - phi[o]) / h : 0.0;",
     "gz[o] = (z < p - 1 && z > 0) ? (phi[o] - phi[ID4(i, j, z - 1, c, n, p, k)]) / h : 0.0;"),
    ("u_z extrapolation dropped", "bz[s] = 2.0 * uz1[s] - uz[s];", "bz[s] = uz1[s];"),
    ("2-D step rule on the 3-D grid", "if (q->mu <= 0.0) q->mu = q->h * q->h / (48.0 * q->tau);",
     "if (q->mu <= 0.0) q->mu = q->h * q->h / (32.0 * q->tau);"),
    ("u_z left out of the objective", "s += sqrt(bx[c] * bx[c] + by[c] * by[c] + bz[c] * bz[c]);",
     "s += sqrt(bx[c] * bx[c] + by[c] * by[c]);"),
    ("y and z swapped in the gradient", "gy[o] = j < n - 1 ? (phi[ID4(i, j + 1, z, c, n, p, k)] - phi[o]) / h : 0.0;",
     "gy[o] = (j < n - 1 && z < p - 1) ? (phi[ID4(i, j, z + 1, c, n, p, k)] - phi[o]) / h : 0.0;"),
]


@pytest.mark.skipif(shutil.which("gcc") is None, reason="needs gcc")
@pytest.mark.parametrize("name,old,new", GRID3_MUTANTS, ids=[m[0] for m in GRID3_MUTANTS])
def test_grid3_pins_reject_mutant(tmp_path, name, old, new):
    src = open(SRC3).read()
    assert old in src, f"pattern for '{name}' not found"
    mut = tmp_path / "mut.c"
    mut.write_text(src.replace(old, new, 1))
    so = tmp_path / "libmut.so"
    subprocess.run(["gcc", "-O2", "-std=c99", "-fPIC", "-shared", "-ffp-contract=off", "-o", str(so), SRC, str(mut),
                    "-lm"], check=True)
    env = dict(os.environ, OMT_ORACLE_LIB=str(so))
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle3_pins.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant '{name}' survived the pins:\n{r.stdout[-2000:]}"
