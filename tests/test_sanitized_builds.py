"""The CPU oracle and the library's host-side runtime built with
AddressSanitizer and UndefinedBehaviorSanitizer (host code only; no GPU is
touched) and run on dense and ragged states: no memory error, leak or
undefined behaviour. The oracle runs whole steps, fractions, curvatures and
the interface consumers; the runtime its host-only calls (workspace sizes,
argument validation of every entry point, the strings)."""
import os
import shutil
import subprocess

import numpy as np
import pytest

from paper_2309_00338_amd import inputs as I

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g", "-O1"]


def _have(tool):
    return shutil.which(tool) is not None


def _write(d, st, u, v):
    st.c.astype(np.uint8).tofile(os.path.join(d, "c.u8"))
    st.cc.astype(np.uint8).tofile(os.path.join(d, "cc.u8"))
    st.hoff.astype(np.float64).tofile(os.path.join(d, "hoff.f64"))
    st.voff.astype(np.float64).tofile(os.path.join(d, "voff.f64"))
    np.ascontiguousarray(u, np.float64).tofile(os.path.join(d, "u.f64"))
    np.ascontiguousarray(v, np.float64).tofile(os.path.join(d, "v.f64"))


@pytest.mark.skipif(not _have("gcc"), reason="gcc not found")
def test_oracle_under_address_and_undefined_sanitizers(tmp_path):
    exe = str(tmp_path / "drv")
    subprocess.run(["gcc", "-std=c99", "-ffp-contract=off", *SAN, "-o", exe, os.path.join(HERE, "sanitize_driver.c"),
                    os.path.join(ROOT, "oracle", "ebit_oracle.c"), "-lm"], check=True)
    cases = []
    w = I.single_vortex(64, period=2.0, cfl=0.5)
    cases.append(("vortex64", w.state, w.u, w.v, w.dts[0], 6))
    st = I.random_colouring(37, 23, seed=3)
    u, v = I.shear_faces(37, 23, 4)
    cases.append(("dense37x23", st, u, v, 0.45 * st.h / max(np.abs(u).max(), np.abs(v).max()), 4))
    st = I.checkerboard(16, 16, seed=5)
    u, v = I.shear_faces(16, 16, 6)
    cases.append(("checker16", st, u, v, 0.2 * st.h / max(np.abs(u).max(), np.abs(v).max()), 3))
    st = I.init_state(4, 4, [I.Circle(2.1, 1.9, 1.3)], h=0.25)
    u, v = I.uniform_faces(4, 4, 0.4, -0.2)
    cases.append(("tiny4", st, u, v, 0.125, 2))  # 0.2 and 0.1 cells per sweep, away from the walls
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=0", UBSAN_OPTIONS="print_stacktrace=1")
    for name, st, u, v, dt, steps in cases:
        d = tmp_path / name
        d.mkdir()
        _write(str(d), st, u, v)
        r = subprocess.run([exe, str(d), str(st.nx), str(st.ny), repr(st.h), repr(dt), str(steps)], env=env,
                           capture_output=True, text=True, timeout=300)
        assert r.returncode == 0 and "ERROR" not in r.stderr and "runtime error" not in r.stderr, (name, r.stderr[-3000:])
        assert r.stdout.startswith("markers")


HOST_DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "ebit.h"
int main(void) {
  size_t b = 0;
  ebit_grid g = {37, 53, 1.0 / 53, 0};
  if (ebit_workspace_bytes(&g, &b) || b == 0) return 3;
  ebit_grid gs[3] = {{64, 64, 1.0 / 64, 0}, {17, 90, 1.0 / 90, 1}, {300, 6, 1.0 / 300, 2}};
  if (ebit_batch_workspace_bytes(3, gs, &b) || b == 0) return 4;
  uint32_t t = 0;
  if (ebit_pool_grid_bytes(&g, &b, &t) || t == 0) return 5;
  if (ebit_pool_workspace_bytes(8, 1024, 1 << 20, &b)) return 6;
  /* argument errors come back before any device work */
  ebit_grid bad = {3, 64, 1.0, 0};
  if (ebit_workspace_bytes(&bad, &b) != EBIT_ERR_ARG) return 7;
  bad.nx = 64; bad.h = -1.0;
  if (ebit_workspace_bytes(&bad, &b) != EBIT_ERR_ARG) return 8;
  ebit_handle *h = 0;
  if (ebit_create(&g, 0, (void *)256, b, 0, &h) != EBIT_ERR_ARG || h) return 9;
  size_t n = (size_t)(g.nx + 1) * (g.ny + 1);
  unsigned char *c = (unsigned char *)calloc(n, 1), *cc = (unsigned char *)calloc((size_t)g.nx * g.ny, 1);
  double *ho = (double *)calloc((size_t)g.nx * (g.ny + 1), 8), *vo = (double *)calloc((size_t)(g.nx + 1) * g.ny, 8);
  c[5] = 2;  /* not a colour */
  ebit_state s = {c, cc, ho, vo};
  if (ebit_create(&g, &s, (void *)256, 1u << 30, 0, &h) != EBIT_ERR_ARG) return 10;
  c[5] = 1;  /* a marker edge with an offset outside [0, 1] */
  ho[4] = 1.5;
  if (ebit_create(&g, &s, (void *)256, 1u << 30, 0, &h) != EBIT_ERR_ARG) return 11;
  if (ebit_create(&g, &s, (void *)255, 1u << 30, 0, &h) != EBIT_ERR_ARG) return 12;  /* misaligned */
  if (ebit_advect(0, 0, 0, 1.0) != EBIT_ERR_ARG || ebit_sync(0) != EBIT_ERR_ARG) return 13;
  ebit_batch *bb = 0;
  if (ebit_batch_create(0, gs, 0, 0, 0, 0, &bb) != EBIT_ERR_ARG) return 14;
  ebit_pool *pp = 0;
  if (ebit_pool_create(0, 1, (void *)256, 1, 0, &pp) != EBIT_ERR_ARG) return 15;
  ebit_graph *gr = 0;
  if (ebit_batch_capture(0, 4, 0, 0, 0, 0, 0, &gr) != EBIT_ERR_ARG) return 16;
  ebit_grid big = {4000, 4000, 1e-3, 0};
  if (ebit_step_static(&big, (unsigned char *)16, (unsigned char *)16, (double *)16, (double *)16, (double *)16,
                       (double *)16, 1e-3, 0, (double *)16, (double *)16, (int32_t *)16, 0) != EBIT_ERR_NOMEM) return 17;
  ebit_schedule sc = {0, 0, 0, -1.0, 0.0};
  if (ebit_set_schedule(0, &sc) != EBIT_ERR_ARG) return 18;
  for (int k = -1; k < 9; k++) if (!ebit_strerror(k) || !strlen(ebit_strerror(k))) return 19;
  free(c); free(cc); free(ho); free(vo);
  printf("host ok\n");
  return 0;
}
"""


@pytest.mark.skipif(not _have("hipcc"), reason="hipcc not found")
def test_runtime_host_code_under_address_and_undefined_sanitizers(tmp_path):
    drv = tmp_path / "host_driver.cpp"
    drv.write_text(HOST_DRIVER)
    exe = str(tmp_path / "host")
    csrc = os.path.join(ROOT, "paper_2309_00338_amd", "csrc")
    host_san = []
    for f in SAN:
        host_san += ["-Xarch_host", f] if f.startswith("-fsanitize") or f.startswith("-fno-sanitize") else [f]
    subprocess.run(["hipcc", "--offload-arch=gfx950", "-std=c++17", "-ffp-contract=off", *host_san,
                    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
                    "-I", os.path.join(ROOT, "include"), "-I", csrc, "-o", exe,
                    os.path.join(csrc, "ebit_kernels.hip"), os.path.join(csrc, "ebit_runtime.hip"), str(drv)],
                   check=True, capture_output=True)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0", UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([exe], env=env, capture_output=True, text=True, timeout=300)
    assert r.returncode == 0 and "runtime error" not in r.stderr and "ERROR: AddressSanitizer" not in r.stderr, \
        (r.returncode, r.stdout[-2000:], r.stderr[-3000:])
