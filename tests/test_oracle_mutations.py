"""Planted mistakes in the oracle must be caught by its pins.

Each case edits one line of a copy of oracle.c (the kind of slip a reader could
make when writing eq. 1-4 down), builds it on the CPU, and runs the pin suite
against it in a subprocess: the suite has to fail. This guards the claim that
the pins constrain every term of the oracle.
"""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "oracle.c")

MUTANTS = {
    "deflection-sign": ("*y1 = a1 * x1 - alpha1;", "*y1 = a1 * x1 + alpha1;"),
    "r-not-squared": ("const double q = m / r2;", "const double q = m / sqrt(r2);"),
    "mass-ignored": ("const double q = m / r2;", "const double q = 1.0 / r2;"),
    "sheet-dropped": ("const double a1 = (1.0 - gamma) - kappa_s;       /* eq. 1, x1 diagonal */",
                      "const double a1 = (1.0 - gamma);"),
    "shear-sign": ("const double a2 = (1.0 + gamma) - kappa_s;       /* eq. 1, x2 diagonal */",
                   "const double a2 = (1.0 - gamma) - kappa_s;"),
    "kappa-not-s-kappa": ("const double kappa_s = s * kappa;                /* eq. 2 */",
                          "const double kappa_s = kappa;"),
    "lens-coords-swapped": ("const double d2 = x2 - lx2[k];", "const double d2 = x2 - lx1[k];"),
    "ray-not-cell-centred": ("const double x1 = base1 + ((double)i + 0.5) * d1;",
                             "const double x1 = base1 + ((double)i) * d1;"),
    "pixel-index-transposed": ("return iy * (int64_t)p1 + ix;", "return ix * (int64_t)p2 + iy;"),
    "upper-edge-closed": ("if (!(u1 >= 0.0 && u1 < (double)p1)) return -1;",
                          "if (!(u1 >= 0.0 && u1 <= (double)p1)) return -1;"),
    "n-avg-factor": ("const double ray_density = ((double)n1 * (double)n2) / (4.0 * h1 * h2);",
                     "const double ray_density = ((double)n1 * (double)n2) / (2.0 * h1 * h2);"),
    "mpd-scale-without-mu-ref": ("const double scale = n_avg * mu_ref;", "const double scale = n_avg;"),
    "mpd-edge-closed": ("while (b <= nbins && thr[b] <= c) ++b;", "while (b <= nbins && thr[b] < c) ++b;"),
    "mpd-values-edge-closed": ("while (b <= nbins && thr[b] <= mu[k]) ++b;",
                               "while (b <= nbins && thr[b] < mu[k]) ++b;"),
    "mpd-values-overflow-dropped": ("while (b <= nbins && thr[b] <= mu[k]) ++b;",
                                    "while (b < nbins && thr[b] <= mu[k]) ++b;"),
    "probability-sum-closed": ("if ((double)counts[k] / n_avg < mu_lim) lo += 1;",
                               "if ((double)counts[k] / n_avg <= mu_lim) lo += 1;"),
    "histogram-overflow-dropped": ("hist[c < n_values - 1 ? c : n_values - 1] += 1;",
                                   "if (c < n_values - 1) hist[c] += 1;"),
    "codec-bits-off-by-one": ("while (b < 32 && ((int64_t)1 << b) < nd) ++b;",
                              "while (b < 32 && ((int64_t)1 << b) <= nd) ++b;"),
    "codec-unsorted-index": ("qsort(values, (size_t)n_pix, sizeof(int32_t), cmp_i32);", ""),
    "normalise-float32-division": ("mu[k] = (float)((double)counts[k] / n_avg);",
                                   "mu[k] = (float)counts[k] / (float)n_avg;"),
    "normalise-reciprocal-multiply": ("mu[k] = (float)((double)counts[k] / n_avg);",
                                      "mu[k] = (float)((double)counts[k] * (1.0 / n_avg));"),
    "normalise-count-through-float": ("mu[k] = (float)((double)counts[k] / n_avg);",
                                      "mu[k] = (float)((float)counts[k] / n_avg);"),
    "row-offset": ("const double x2 = base2 + ((double)j + 0.5) * d2;\n        for (int64_t i = 0; i < n1; ++i) {\n            const double x1 = base1 + ((double)i + 0.5) * d1;\n            double y1, y2;",
                   "const double x2 = base2 + ((double)(j - row_begin) + 0.5) * d2;\n        for (int64_t i = 0; i < n1; ++i) {\n            const double x1 = base1 + ((double)i + 0.5) * d1;\n            double y1, y2;"),
}
# Not listed: dropping the singular-ray test in oracle_shoot changes nothing,
# because a ray exactly on a lens already has a NaN position (0 * inf) and NaN
# fails every window comparison; the pin on singular rays covers both routes.


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_planted_mistake_is_caught(name, tmp_path):
    old, new = MUTANTS[name]
    src = open(SRC).read()
    assert src.count(old) >= 1, f"mutation site for {name} not found"
    mutated = src.replace(old, new)
    (tmp_path / "oracle.h").write_text(open(os.path.join(ROOT, "oracle", "oracle.h")).read())
    c_path = tmp_path / "oracle.c"
    c_path.write_text(mutated)
    lib = tmp_path / "liboracle_mutant.so"
    subprocess.run(["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared",
                    "-o", str(lib), str(c_path), "-lm"], check=True)
    env = dict(os.environ, ORACLE_LIB=str(lib), OMP_NUM_THREADS=os.environ.get("OMP_NUM_THREADS", "4"))
    r = subprocess.run([sys.executable, "-m", "pytest", "-x", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_oracle_pins.py"),
                        os.path.join(ROOT, "tests", "test_oracle_mpd.py"),
                        os.path.join(ROOT, "tests", "test_oracle_codec.py")],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=600)
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"


# Planted mistakes in the Python part of the oracle (finite-source kernels and
# the convolution of Section 2.4, oracle/convolve.py): the mutated module is
# loaded in place of oracle.convolve in a subprocess that runs its pin suite.
CONVOLVE_SRC = os.path.join(ROOT, "oracle", "convolve.py")
PY_MUTANTS = {
    "kernel-subsamples-off-centre": ("off = (np.arange(subsamples) + 0.5) / subsamples - 0.5",
                                     "off = np.arange(subsamples) / subsamples - 0.5"),
    "kernel-pixel-shifted": ("K[j % p2, i % p1] = brightness(", "K[(j + 1) % p2, i % p1] = brightness("),
    "kernel-not-normalised": ("return K / total", "return K"),
    "correlation-not-convolution": ("C = np.fft.ifft2(np.fft.fft2(M) * np.fft.fft2(K)).real",
                                    "C = np.fft.ifft2(np.fft.fft2(M) * np.conj(np.fft.fft2(K))).real"),
    "gaussian-sigma": ("sigma = radius / 3.0", "sigma = radius / 2.0"),
    "power-slope": ("I = (np.maximum(r, core) / radius) ** (-0.75)",
                    "I = (np.maximum(r, core) / radius) ** (-0.5)"),
    "hole-ignored": ("return np.where((r < radius) & (r >= hole), I, 0.0)",
                     "return np.where(r < radius, I, 0.0)"),
    "table-boxes-not-centred": ("ix = np.floor(x / pix1 + 0.5).astype(np.int64)",
                                "ix = np.floor(x / pix1).astype(np.int64)"),
    "table-axes-swapped": ("compact[iy[ky] + h2, ix[kx] + h1] += b[ky, kx]",
                           "compact[iy[ky] + h2, ix[kx] + h1] += b.T.reshape(b.shape)[ky, kx]"),
    "table-not-normalised": ("K[j % p2, i % p1] = compact[j + h2, i + h1] / total",
                             "K[j % p2, i % p1] = compact[j + h2, i + h1]"),
}

_BOOT = """
import importlib.util, sys
sys.path.insert(0, {root!r})
import oracle
spec = importlib.util.spec_from_file_location("oracle.convolve", {path!r})
mod = importlib.util.module_from_spec(spec)
spec.loader.exec_module(mod)
sys.modules["oracle.convolve"] = mod
oracle.convolve = mod
import pytest
sys.exit(pytest.main(["-x", "-q", "-p", "no:cacheprovider", {tests!r}]))
"""


@pytest.mark.parametrize("name", sorted(PY_MUTANTS))
def test_planted_mistake_in_convolution_oracle_is_caught(name, tmp_path):
    old, new = PY_MUTANTS[name]
    src = open(CONVOLVE_SRC).read()
    assert src.count(old) == 1, f"mutation site for {name} not found"
    path = tmp_path / "convolve_mutant.py"
    path.write_text(src.replace(old, new))
    code = _BOOT.format(root=ROOT, path=str(path),
                        tests=os.path.join(ROOT, "tests", "test_oracle_convolve.py"))
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode not in (0, 4, 5), f"bad run for {name}:\n{r.stdout[-2000:]}{r.stderr[-2000:]}"
    assert r.returncode != 0, f"mutant {name} passed every pin:\n{r.stdout[-2000:]}"


def test_unmutated_convolution_oracle_passes_through_the_same_harness(tmp_path):
    """The harness itself: the unchanged module loaded the same way passes."""
    path = tmp_path / "convolve_copy.py"
    path.write_text(open(CONVOLVE_SRC).read())
    code = _BOOT.format(root=ROOT, path=str(path),
                        tests=os.path.join(ROOT, "tests", "test_oracle_convolve.py"))
    r = subprocess.run([sys.executable, "-c", code], cwd=str(tmp_path), capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 0, r.stdout[-2000:] + r.stderr[-2000:]
