"""The boundary from C: include/bartlett.h compiles as C99 with warnings as
errors, and a C program linked against libbartlett.so reaches the entry
points (argument-error paths only, which run without a GPU)."""
import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIBDIR = os.path.join(ROOT, "paper_2604_19723_amd")

PROGRAM = r"""
#include <stdio.h>
#include <string.h>
#include "bartlett.h"

#define CHECK(cond) do { if (!(cond)) { printf("FAIL line %d\n", __LINE__); return 1; } } while (0)

int main(void) {
  size_t sz = 0;
  ba_plan plan = NULL;
  ba_msgs msgs = NULL;
  ba_coherent coh = NULL;
  ba_msg_inputs in;
  ba_msg_outputs out;
  double pos[3] = {0.0, 0.0, 0.0};
  memset(&in, 0, sizeof in);
  memset(&out, 0, sizeof out);
  CHECK(ba_status_string(BA_OK) != NULL);
  CHECK(ba_version() != NULL && strlen(ba_version()) > 0);
  CHECK(ba_plan_create(&plan, 0, pos, BA_GRID_ULA_DEG, 1, pos, 1, 0, 0, BA_PREC_F32) == BA_ERR_ARG);
  CHECK(plan == NULL);
  CHECK(ba_workspace_size(NULL, 1, 1, 1, &sz) == BA_ERR_ARG);
  CHECK(ba_msgs_create(&msgs, 0, pos, pos, 4, 4, 10, 3.5e9, 1e8) == BA_ERR_ARG);
  CHECK(ba_msgs_workspace_size(NULL, 6, 100, &sz) == BA_ERR_ARG);
  CHECK(ba_update_messages(NULL, &in, &out, NULL, 0, NULL) == BA_ERR_ARG);
  CHECK(ba_coherent_destroy(coh) == BA_ERR_ARG);
  CHECK(strlen(ba_last_error()) > 0);
  printf("ok\n");
  return 0;
}
"""


def test_header_compiles_as_c_and_links():
    gcc = shutil.which("gcc")
    if gcc is None:
        pytest.skip("gcc not available")
    lib = os.path.join(LIBDIR, "libbartlett.so")
    if not os.path.exists(lib):
        pytest.skip("libbartlett.so is not built")
    work = os.path.join(ROOT, "_build_c_header")
    os.makedirs(work, exist_ok=True)
    try:
        src = os.path.join(work, "abi.c")
        exe = os.path.join(work, "abi")
        with open(src, "w") as f:
            f.write(PROGRAM)
        cmd = [gcc, "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic", "-I", os.path.join(ROOT, "include"),
               src, "-o", exe, "-L", LIBDIR, "-lbartlett", "-Wl,-rpath," + LIBDIR]
        r = subprocess.run(cmd, capture_output=True, text=True)
        assert r.returncode == 0, r.stderr
        r = subprocess.run([exe], capture_output=True, text=True, timeout=120)
        assert r.returncode == 0 and r.stdout.strip().endswith("ok"), r.stdout + r.stderr
    finally:
        shutil.rmtree(work, ignore_errors=True)
