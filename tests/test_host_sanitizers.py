"""Host code under AddressSanitizer and UndefinedBehaviorSanitizer (no GPU):
the C-ABI translation units are rebuilt with both sanitizers on the host side
and linked with the library's normally built HIP objects; a C driver then runs
argument validation, workspace sizing, a sweep of launch configurations,
ragged batched-plan construction (up to the device allocation, which fails
without a GPU) and the tuning table's text round trip, including malformed
files. Any memory error or undefined behaviour aborts the driver."""
import glob
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2109_05496_amd", "csrc")
BUILD = os.path.join(ROOT, "_build")
ROCM = "/opt/rocm"
HIPCC = os.path.join(ROCM, "bin", "hipcc")
CLANG = os.path.join(ROCM, "llvm", "bin", "clang")
HOST_UNITS = ("capi", "batched", "autotune", "adjoint", "pr")
DEVICE_OBJS = ("fgp_forward.hip.o", "fgp_adjoint.hip.o", "fft_pr.hip.o")
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined"]

pytestmark = [pytest.mark.skipif(not (os.path.exists(HIPCC) and os.path.exists(CLANG)
                                      and all(os.path.exists(os.path.join(BUILD, o)) for o in DEVICE_OBJS)),
                                 reason="needs hipcc, ROCm clang and the library's built objects")]

DRIVER = r"""
#include <stdio.h>
#include <stdlib.h>
#include <string.h>
#include "ctv.h"
static int n_calls = 0;
#define SHOW(x) do { ctv_status s_ = (x); ++n_calls; if (s_) (void)ctv_last_error(); printf("%-40.40s -> %d\n", #x, s_); } while (0)
int main(void) {
  ctv_params p = {sizeof(ctv_params), CTV_TV_1I, 0.5f, CTV_C_MODULUS, 100, 0, 0, 0, CTV_M_FGP, CTV_S_AUTO};
  size_t ws = 0, sv = 0;
  int32_t T, R, W, Pp;
  float lam[40];
  for (int i = 0; i < 40; ++i) lam[i] = 0.05f;
  void* dummy = (void*)0x1000;
  SHOW(ctv_workspace_size(&p, 40, 300, 257, 7, &ws, &sv));
  SHOW(ctv_workspace_size(&p, 0, 8, 8, 0, &ws, &sv));
  for (int k = 0; k < 4; ++k) {
    p.tv_kind = k;
    for (int w = -1; w <= 16; ++w)
      for (int r = 0; r <= 16; ++r) {
        p.tile_waves = w; p.tile_rows = r;
        for (int f = 0; f <= 17; f += 3) { p.fuse = f; (void)ctv_tiling(&p, 1, 1 + 37 * f, 2048, &T, &R, &W, &Pp); }
      }
  }
  p.tile_waves = p.tile_rows = p.fuse = 0;
  p.tv_kind = CTV_TV_1I;
  SHOW(ctv_denoise(&p, 1, 8, 8, NULL, lam, NULL, dummy, NULL, NULL, 0, NULL, 0, NULL, dummy, 1 << 20, NULL));
  SHOW(ctv_denoise(&p, 1, 8, 8, dummy, lam, NULL, dummy, NULL, NULL, 0, NULL, 0, NULL, dummy, 1 << 20, NULL));
  lam[0] = -1.0f;
  SHOW(ctv_denoise(&p, 1, 8, 8, dummy, lam, NULL, (float*)0x2000, NULL, NULL, 0, NULL, 0, NULL, dummy, 1 << 20, NULL));
  lam[0] = 0.05f;
  SHOW(ctv_denoise(&p, 1, 8, 8, dummy, lam, NULL, (float*)0x2000, NULL, NULL, 0, NULL, 0, NULL, dummy, 16, NULL));
  SHOW(ctv_denoise_backward(&p, 1, 8, 8, dummy, lam, NULL, 0, NULL, dummy, dummy, dummy, dummy, 1 << 20, NULL));
  /* batched: ragged descriptors, then the device tables fail to allocate without a GPU */
  ctv_image_desc d[300];
  long long off = 0;
  for (int i = 0; i < 300; ++i) {
    d[i].offset = off; d[i].m = 1 + (i * 37) % 700; d[i].n = 1 + (i * 53) % 900; d[i].lambda = (i % 7) ? 0.05f : 0.0f;
    d[i].tv_kind = i % 4; d[i].alpha = 0.3f; d[i].iters = (i * 13) % 170; d[i].support_offset = (i % 3) ? -1 : off;
    off += (long long)d[i].m * d[i].n;
  }
  ctv_batched_plan* plan = NULL;
  SHOW(ctv_batched_plan_create(d, 300, &p, &plan));
  if (plan) { SHOW(ctv_batched_plan_destroy(plan)); }
  d[5].offset = d[4].offset;
  SHOW(ctv_batched_plan_create(d, 300, &p, &plan));
  int32_t found = 0;
  SHOW(ctv_batched_tune_lookup(d, 300, &p, &found, NULL));
  SHOW(ctv_tune_lookup(&p, 1, 64, 64, &found, NULL));
  /* tune table text */
  FILE* f = fopen("t.jsonl", "w");
  for (int i = 0; i < 50; ++i)
    fprintf(f, "{\"arch\": \"gfx950:x/%dcu/hip1\", \"key\": \"%016x\", \"fuse\": %d, \"tile_waves\": 8, \"tile_rows\": %d, \"ms\": 1.5, \"what\": \"entry %d\"}\n", i, i * 7919, 1 + i % 16, (i % 2) ? 4 : 8, i);
  fprintf(f, "\n   \n");
  fclose(f);
  SHOW(ctv_tune_cache_load("t.jsonl"));
  printf("size %d\n", ctv_tune_cache_size());
  SHOW(ctv_tune_cache_save("t2.jsonl"));
  SHOW(ctv_tune_cache_load("t2.jsonl"));
  printf("size %d\n", ctv_tune_cache_size());
  f = fopen("bad.jsonl", "w");
  fprintf(f, "{\"arch\": \"a\", \"key\": \"zz\", \"fuse\": 3}\n{\"arch\": \"");
  fclose(f);
  SHOW(ctv_tune_cache_load("bad.jsonl"));
  f = fopen("bad2.jsonl", "w");
  fprintf(f, "{\"arch\": \"a\", \"key\": \"12\", \"fuse\": 1e400, \"tile_waves\": 8, \"tile_rows\": 8, \"ms\": 1}\n");
  fclose(f);
  SHOW(ctv_tune_cache_load("bad2.jsonl"));
  f = fopen("bad3.jsonl", "w");
  fprintf(f, "{\"arch\": \"a\", \"key\": \"12\", \"fuse\": 3, \"tile_waves\": 99999999999, \"tile_rows\": 8, \"ms\": 1}\n");
  fclose(f);
  SHOW(ctv_tune_cache_load("bad3.jsonl"));
  SHOW(ctv_tune_cache_clear());
  ctv_tuning res[4];
  SHOW(ctv_autotune(&p, 1, 64, 64, dummy, lam, NULL, dummy, dummy, 1 << 20, 0, res, 4, NULL, NULL, NULL));
  /* phase retrieval argument checks */
  double dist[4] = {1e-3, 1.5e-3, 2e-3, 2.5e-3};
  pr_params pp;
  memset(&pp, 0, sizeof(pp));
  pp.struct_size = sizeof(pr_params); pp.num_meas = 4; pp.distances_host = dist; pp.wavelength = 532e-9;
  pp.pixel = 4e-6; pp.tau = 0.01f; pp.gamma = 0.25f; pp.outer_iters = 10; pp.inner = p; pp.inner.iters = 20;
  pp.init_backprop = 1; pp.accelerate = 1; pp.ls_shrink = 0.5f; pp.ls_max_trials = 5;
  SHOW(pr_workspace_size(&pp, 1024, 1024, &ws));
  SHOW(pr_workspace_size(&pp, 1000, 1024, &ws));
  SHOW(pr_workspace_size(&pp, 4096, 2, &ws));
  SHOW(pr_prox_grad(&pp, 64, 64, NULL, dummy, NULL, NULL, dummy, 1 << 30, NULL));
  pp.num_meas = 0;
  SHOW(pr_workspace_size(&pp, 64, 64, &ws));
  SHOW(ctv_fft2_workspace_size(3, 256, 2048, &ws));
  SHOW(ctv_fft2_workspace_size(3, 255, 2048, &ws));
  printf("calls %d done\n", n_calls);
  return 0;
}
"""

EXPECTED = {
    "ctv_workspace_size(&p, 40, 300, 257, 7,": "0", "ctv_workspace_size(&p, 0, 8, 8, 0, &ws,": "-1",
    "ctv_batched_plan_create(d, 300, &p, &pla": None, "ctv_tune_cache_load(\"t.jsonl\")": "0",
    "ctv_tune_cache_load(\"bad.jsonl\")": "-1", "ctv_tune_cache_load(\"bad2.jsonl\")": "-1",
    "ctv_tune_cache_load(\"bad3.jsonl\")": "-1", "pr_workspace_size(&pp, 1000, 1024, &ws)": "-4",
}


def test_host_code_under_asan_and_ubsan(tmp_path):
    def run(cmd, **kw):
        r = subprocess.run(cmd, capture_output=True, text=True, **kw)
        assert r.returncode == 0, " ".join(cmd) + "\n" + r.stdout[-3000:] + r.stderr[-3000:]
        return r

    flags = ["-O1", "-g", "-std=c++17", "-fPIC", "-ffp-contract=off", "-fno-omit-frame-pointer",
             "-I" + os.path.join(ROOT, "include"), "-I" + CSRC, "-x", "c++", "-D__HIP_PLATFORM_AMD__",
             "-I" + ROCM + "/include"]
    procs = [subprocess.Popen([HIPCC] + flags + SAN + ["-c", os.path.join(CSRC, u + ".cpp"), "-o",
                                                        str(tmp_path / (u + ".o"))],
                              stdout=subprocess.PIPE, stderr=subprocess.PIPE, text=True) for u in HOST_UNITS]
    for p in procs:
        out, err = p.communicate()
        assert p.returncode == 0, err[-3000:]
    lib = tmp_path / "libctv_san.so"
    run([HIPCC, "--offload-arch=gfx950", "-shared", "-fPIC"] + SAN + ["-o", str(lib)]
        + [str(tmp_path / (u + ".o")) for u in HOST_UNITS] + [os.path.join(BUILD, o) for o in DEVICE_OBJS])
    (tmp_path / "drv.c").write_text(DRIVER)
    exe = tmp_path / "drv"
    run([CLANG, "-std=c99", "-g", "-fsanitize=address,undefined", "-fno-omit-frame-pointer", "-shared-libsan",
         "-I" + os.path.join(ROOT, "include"), str(tmp_path / "drv.c"), "-o", str(exe), "-L" + str(tmp_path),
         "-lctv_san", "-Wl,-rpath," + str(tmp_path), "-Wl,-rpath-link," + ROCM + "/lib"])
    rt = glob.glob(os.path.join(ROCM, "llvm", "lib", "clang", "*", "lib", "linux", "libclang_rt.asan-x86_64.so"))
    assert rt, "sanitizer runtime not found"
    env = dict(os.environ, LD_LIBRARY_PATH=os.path.dirname(rt[0]), ASAN_OPTIONS="detect_leaks=0:halt_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, cwd=tmp_path, env=env, timeout=300)
    assert r.returncode == 0, r.stdout[-3000:] + r.stderr[-3000:]
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr[-3000:]
    lines = {l[:40].rstrip(): l.rsplit("->", 1)[1].strip() for l in r.stdout.splitlines() if "->" in l}
    for call, status in EXPECTED.items():
        assert call in lines, call
        if status is not None:
            assert lines[call] == status, (call, lines[call])
    assert lines["ctv_batched_plan_create(d, 300, &p, &pla"] != "0"
    assert "size 50" in r.stdout and "done" in r.stdout
