"""The oracle's pins have teeth: each plausible mistake planted in a copy of
the oracle source (on the CPU) must make at least one pin test fail."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "nbody_oracle.c")
PINS = ["tests/test_oracle_accel.py", "tests/test_oracle_halo.py",
        "tests/test_oracle_integrators.py", "tests/test_oracle_diag.py", "tests/test_oracle_density.py",
        "tests/test_oracle_hermite.py"]

# (name, original text, planted mistake); each original occurs in the source
MUTATIONS = [
    ("softening dropped", "const double d2 = eps * eps;\n    double ax = 0.0", "const double d2 = 0.0 * eps;\n    double ax = 0.0"),
    ("jerk softening dropped", "const double d2 = eps * eps;\n    double ax = 0, ay", "const double d2 = 0.0 * eps;\n    double ax = 0, ay"),
    ("attraction sign", "ax -= s * dx;", "ax += s * dx;"),
    ("source mass index", "const double s = G * m[j] / r3;", "const double s = G * m[i] / r3;"),
    ("distance power", "const double r3 = r2 * r;", "const double r3 = r2;"),
    ("transposed coordinate", "const double dz = z[i] - z[j];\n        const double r2 = dx * dx + dy * dy + dz * dz + d2;\n        if (r2 == 0.0) continue;                    /* zero",
     "const double dz = y[i] - y[j];\n        const double r2 = dx * dx + dy * dy + dz * dz + d2;\n        if (r2 == 0.0) continue;                    /* zero"),
    ("self pair kept", "if (j == i) continue;                       /* Eq. (1): j != i */", ""),
    ("half-step drift", "x[i] += dt * vx[i];", "x[i] += dt / 2.0 * vx[i];"),
    ("paper-form corrector", "vx[i] = (vx[i] + wx) / 2.0;", "vx[i] = wx;"),
    ("fourth-order middle weight", "h, w0 * dt, 0,", "h, w1 * dt, 0,"),
    ("potential energy double count", "W -= w[i] / 2.0;", "W -= w[i];"),
    ("kinetic energy factor", "vz[i] * vz[i]) / 2.0;", "vz[i] * vz[i]);"),
    ("angular momentum cross product", "L[2] += m[i] * (x[i] * vy[i] - y[i] * vx[i]);", "L[2] += m[i] * (x[i] * vx[i] - y[i] * vy[i]);"),
    ("halo field power", "return v2 * (1.0 - atan(s) / s) / (r * r);", "return v2 * (1.0 - atan(s) / s) / r;"),
    ("halo potential log factor", "return v2 * (atan_over_s + 0.5 * log1p(s * s));", "return v2 * (atan_over_s + log1p(s * s));"),
    ("halo core series", "sum += ((k % 2) ? term : -term) / (2.0 * k + 1.0);", "sum += term / (2.0 * k + 1.0);"),
    ("jerk radial term sign", "jx += G * m[j] * (ux / R3 - 3.0 * rv * rx / R5);", "jx += G * m[j] * (ux / R3 + 3.0 * rv * rx / R5);"),
    ("jerk relative velocity", "const double ux = vx[j] - vx[i], uy", "const double ux = vx[j] + vx[i], uy"),
    ("halo jerk radial term dropped", "o[3] -= g * vx[i] + hh * rv * x[i];", "o[3] -= g * vx[i];"),
    ("halo jerk series sign", "sum += ((k % 2) ? term : -term) * (2.0 * k - 2.0) / (2.0 * k + 1.0);", "sum += term * (2.0 * k - 2.0) / (2.0 * k + 1.0);"),
    ("hermite position corrector", "x[i] += (vx[i] + wx) * dt / 2.0 + (ax[i] - bx[i]) * dt * dt / 12.0;", "x[i] += (vx[i] + wx) * dt / 2.0;"),
    ("hermite velocity corrector", "const double wy = vy[i] + (ay[i] + by[i]) * dt / 2.0 + (jy[i] - ky[i]) * dt * dt / 12.0;", "const double wy = vy[i] + (ay[i] + by[i]) * dt / 2.0 + (jy[i] - ky[i]) * dt * dt / 6.0;"),
    ("hermite predictor without jerk", "py[i] = y[i] + vy[i] * dt + ay[i] * dt * dt / 2.0 + jy[i] * dt * dt * dt / 6.0;", "py[i] = y[i] + vy[i] * dt + ay[i] * dt * dt / 2.0;"),
    ("rk4 weight", "y[i] += dt / 6.0 * (k1ry[i] + 2.0 * k2ry[i] + 2.0 * k3ry[i] + k4ry[i]);", "y[i] += dt / 6.0 * (k1ry[i] + 2.0 * k2ry[i] + k3ry[i] + 2.0 * k4ry[i]);"),
    ("rk4 last stage", "sy[i] = y[i] + dt * k3ry[i];", "sy[i] = y[i] + dt / 2.0 * k3ry[i];"),
    ("density map transposed", "counts[(int64_t)fy * nx + (int64_t)fx] += 1u;", "counts[(int64_t)fx * ny + (int64_t)fy] += 1u;"),
    ("density right edge kept", "fx < (double)nx && fy", "fx <= (double)nx && fy"),
    ("density cell scale", "const double fy = floor((y[i] - y0) * sy);", "const double fy = floor((y[i] - y0) * sx);"),
    ("halo series branch point", "if (s < 0.5) return v2 / (rc * rc) * halo_series_over_s2(s);", "if (s < 0.5) return v2 / (rc * rc) / 3.0;"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,bad", MUTATIONS, ids=[m[0] for m in MUTATIONS])
def test_pins_catch_planted_mistake(tmp_path, name, orig, bad):
    import oracle
    text = open(SRC).read()
    assert text.count(orig) == 1, f"mutation anchor not unique: {name}"
    src = tmp_path / "mut.c"
    src.write_text(text.replace(orig, bad))
    lib = oracle.build(force=True, src=str(src), out=str(tmp_path / "libmut.so"))
    env = dict(os.environ, NBODY_ORACLE_LIB=lib, OMP_NUM_THREADS="4")
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        *PINS], cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"no pin caught the planted mistake: {name}\n{r.stdout[-2000:]}"


METRICS_SRC = os.path.join(ROOT, "oracle", "metrics.py")

# planted mistakes in the force-error metrics (oracle/metrics.py)
METRICS_MUTATIONS = [
    ("conditioned error: mean for max", "\"eps_cond\": float(np.max(d[A > 0] / A[A > 0]))",
     "\"eps_cond\": float(np.mean(d[A > 0] / A[A > 0]))"),
    ("difference norm over the wrong axis", "d = np.sqrt(((got - ref) ** 2).sum(0))",
     "d = np.sqrt(((got - ref) ** 2).sum(1))"),
    ("dropped square root", "d = np.sqrt(((got - ref) ** 2).sum(0))", "d = ((got - ref) ** 2).sum(0)"),
]


@pytest.mark.slow
@pytest.mark.parametrize("name,orig,bad", METRICS_MUTATIONS, ids=[m[0] for m in METRICS_MUTATIONS])
def test_metric_pins_catch_planted_mistake(tmp_path, name, orig, bad):
    text = open(METRICS_SRC).read()
    assert text.count(orig) == 1, f"mutation anchor not unique: {name}"
    src = tmp_path / "metrics_mut.py"
    src.write_text(text.replace(orig, bad))
    env = dict(os.environ, NBODY_METRICS_SRC=str(src))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_metrics.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0, f"no pin caught the planted mistake: {name}\n{r.stdout[-2000:]}"


EQ_SRC = os.path.join(ROOT, "oracle", "equilibrium.py")

# planted mistakes in the disk-equilibrium reference (oracle/equilibrium.py)
EQ_MUTATIONS = [
    ("rho_* sign", "return w, -k4 * (math.exp(u) - rho_star)", "return w, -k4 * (math.exp(u) + rho_star)"),
    ("4 pi G factor", "k4 = 4.0 * math.pi * G / cz2", "k4 = 2.0 * math.pi * G / cz2"),
    ("RK4 weights", "u_new = u + h / 6.0 * (a1 + 2.0 * a2 + 2.0 * a3 + a4)",
     "u_new = u + h / 4.0 * (a1 + a2 + a3 + a4)"),
    ("column without both sides", "    return 2.0 * s", "    return s"),
    ("drift term sign", "out.append(vc2[k] + cr2[k] * (1.0 - cphi2[k] / cr2[k] + dlog))",
     "out.append(vc2[k] + cr2[k] * (1.0 - cphi2[k] / cr2[k] - dlog))"),
    ("dispersion ratio dropped", "out.append(vc2[k] + cr2[k] * (1.0 - cphi2[k] / cr2[k] + dlog))",
     "out.append(vc2[k] + cr2[k] * (1.0 + dlog))"),
    ("log derivative in r", "/ (math.log(r[b]) - math.log(r[a]))", "/ (r[b] - r[a])"),
]


@pytest.mark.parametrize("name,orig,bad", EQ_MUTATIONS, ids=[m[0] for m in EQ_MUTATIONS])
def test_equilibrium_pins_catch_planted_mistake(tmp_path, name, orig, bad):
    text = open(EQ_SRC).read()
    assert text.count(orig) == 1, f"mutation anchor not unique: {name}"
    src = tmp_path / "equilibrium_mut.py"
    src.write_text(text.replace(orig, bad))
    env = dict(os.environ, NBODY_EQUILIBRIUM_SRC=str(src))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        "tests/test_oracle_equilibrium.py"], cwd=ROOT, env=env, capture_output=True, text=True,
                       timeout=300)
    assert r.returncode != 0, f"no pin caught the planted mistake: {name}\n{r.stdout[-2000:]}"
