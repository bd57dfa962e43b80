"""The C part of the oracle under the compilers' sanitizers (host code only).

- AddressSanitizer and UndefinedBehaviorSanitizer: ``oracle/siddon.c`` built
  with gcc and both sanitizers, driven through the forward projection, the
  scatter adjoint and the nonzero count on a small geometry with odd sizes,
  offsets and anisotropic voxels; any report aborts the run.
- ThreadSanitizer on the OpenMP paths (the adjoint's per-thread partial
  volumes, the forward's ray loop): built with the LLVM OpenMP runtime, whose
  synchronisation the archer tool describes to TSan, so that only races in
  the oracle's own code are reported.  A copy of the oracle with a planted
  race (every thread scattering into one shared volume) must be reported,
  which shows the check can fail.

The driver also checks the adjoint identity, so a sanitizer build that
computed something else would fail too.
"""
import os
import re
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SIDDON = os.path.join(ROOT, "oracle", "siddon.c")
LLVM = "/opt/rocm/llvm"
CLANG = os.path.join(LLVM, "bin", "clang")
ARCHER = os.path.join(LLVM, "lib", "libarcher.so")

DRIVER = r"""
#include <math.h>
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
typedef struct {
    int32_t nx, ny, nz; double vx, vy, vz; double ox, oy, oz;
    int32_t nu, nv; double du, dv; double dso, dsd; int32_t na; const double *angles;
} ora_geom;
int ora_forward(const ora_geom *g, const double *x, double *y);
int ora_adjoint(const ora_geom *g, const double *y, double *x);
int ora_count_nnz(const ora_geom *g, int64_t *nnz, int64_t *hit_rays);
int main(void)
{
    double ang[7];
    for (int a = 0; a < 7; ++a) ang[a] = 6.283185307179586 * a / 7.0 + 0.1;
    ora_geom g = {11, 9, 7, 1.0, 1.1, 0.9, 0.3, -0.2, 0.1, 17, 13, 1.2, 1.0, 60.0, 100.0, 7, ang};
    size_t nv = 11 * 9 * 7, np = 7 * 17 * 13;
    double *x = malloc(nv * sizeof(double)), *y = malloc(np * sizeof(double));
    double *w = malloc(np * sizeof(double)), *z = malloc(nv * sizeof(double));
    for (size_t i = 0; i < nv; ++i) x[i] = (double)((i * 7919) % 101) / 101.0;
    for (size_t i = 0; i < np; ++i) w[i] = (double)((i * 104729) % 97) / 97.0;
    int e = ora_forward(&g, x, y) | ora_adjoint(&g, w, z);
    int64_t nnz = 0, hits = 0;
    e |= ora_count_nnz(&g, &nnz, &hits);
    double lhs = 0.0, rhs = 0.0, ny = 0.0, nw = 0.0;
    for (size_t i = 0; i < np; ++i) { lhs += y[i] * w[i]; ny += y[i] * y[i]; nw += w[i] * w[i]; }
    for (size_t i = 0; i < nv; ++i) rhs += x[i] * z[i];
    double rel = fabs(lhs - rhs) / sqrt(ny * nw);
    printf("status %d nnz %lld hits %lld adjoint %.3e\n", e, (long long)nnz, (long long)hits, rel);
    free(x); free(y); free(w); free(z);
    return (e || nnz <= 0 || rel > 1e-13) ? 3 : 0;
}
"""


def _build(tmp_path, cc, flags, src=SIDDON, name="drv"):
    drv = tmp_path / "driver.c"
    drv.write_text(DRIVER)
    exe = tmp_path / name
    cmd = [cc, "-O1", "-g", "-std=c99", "-ffp-contract=off", "-fopenmp", *flags, str(src), str(drv), "-lm",
           "-o", str(exe)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    return exe


def _run(exe, env_extra):
    env = dict(os.environ, OMP_NUM_THREADS="4", **env_extra)
    return subprocess.run([str(exe)], capture_output=True, text=True, env=env, timeout=120)


def test_oracle_asan_ubsan(tmp_path):
    if shutil.which("gcc") is None:
        pytest.skip("gcc not available")
    exe = _build(tmp_path, "gcc", ["-fsanitize=address,undefined", "-fno-sanitize-recover=all",
                                   "-fno-omit-frame-pointer"])
    r = _run(exe, {"ASAN_OPTIONS": "detect_leaks=1:abort_on_error=0"})
    assert r.returncode == 0, r.stdout + r.stderr
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
    assert re.search(r"status 0 nnz \d+", r.stdout)


def _tsan(tmp_path, src, name):
    if not (os.path.exists(CLANG) and os.path.exists(ARCHER)):
        pytest.skip("LLVM clang with the archer OpenMP tool not available")
    exe = _build(tmp_path, CLANG, ["-fsanitize=thread", f"-Wl,-rpath,{LLVM}/lib"], src=src, name=name)
    return _run(exe, {"OMP_TOOL_LIBRARIES": ARCHER,
                      "TSAN_OPTIONS": "ignore_noninstrumented_modules=1:halt_on_error=1:exitcode=66"})


def test_oracle_openmp_tsan_clean(tmp_path):
    r = _tsan(tmp_path, SIDDON, "tsan")
    assert r.returncode == 0, r.stdout + r.stderr
    assert "ThreadSanitizer" not in r.stderr
    assert "status 0" in r.stdout


def test_tsan_reports_a_planted_race(tmp_path):
    src = open(SIDDON).read()
    planted = src.replace("double *acc = part + (size_t)tid * (size_t)nvox;", "double *acc = part;")
    assert planted != src, "the adjoint's per-thread volume line moved; update the planted race"
    bad = tmp_path / "siddon_race.c"
    bad.write_text(planted)
    r = _tsan(tmp_path, bad, "tsan_race")
    assert r.returncode != 0 and "data race" in r.stderr
