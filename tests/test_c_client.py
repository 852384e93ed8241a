"""The C ABI from plain C (no GPU): svbatch.h compiles as C99 with warnings
as errors, a C program links against libsvbatch.so, and the calls that need
no device behave as the header states: handle creation, options,
validation of circuits and noise models (SV_EINVAL before any device
work), the attach requirement (SV_ESTATE), and the thread-local message."""
import os
import shutil
import subprocess

import pytest

import paper_2308_03399_amd as S

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

C_SOURCE = r"""
#include <stdio.h>
#include <string.h>
#include "svbatch.h"

#define CHECK(cond) do { if (!(cond)) { printf("FAIL line %d\n", __LINE__); return 1; } } while (0)

int main(void)
{
    sv_batch *b = NULL;
    CHECK(sv_batch_create(0, 10, SV_C64, &b) == SV_EINVAL);
    CHECK(sv_batch_create(4, 0, SV_C64, &b) == SV_EINVAL);
    CHECK(sv_batch_create(4, 10, SV_C64, &b) == SV_OK && b != NULL);
    CHECK(sv_batch_set_option(b, "mode", SV_MODE_BRANCH) == SV_OK);
    CHECK(sv_batch_set_option(b, "no_such_option", 1) == SV_EINVAL);
    CHECK(strstr(sv_last_error(), "no_such_option") != NULL);

    /* H on qubit 0, CX 0 -> 3, measure all; one depolarizing rule on H */
    sv_op ops[3];
    memset(ops, 0, sizeof ops);
    ops[0].kind = SV_OP_H; ops[0].nq = 1; ops[0].q[0] = 0;
    ops[1].kind = SV_OP_CX; ops[1].nq = 2; ops[1].q[0] = 0; ops[1].q[1] = 3;
    ops[2].kind = SV_OP_MEASURE; ops[2].nq = 4;
    for (int t = 0; t < 4; ++t) { ops[2].q[t] = (uint32_t)t; ops[2].c[t] = (uint32_t)t; }
    double prob[4] = {0.97, 0.01, 0.01, 0.01};
    uint8_t pauli[4] = {0, 1, 2, 3};
    sv_pauli_channel ch = {1, 4, prob, pauli};
    sv_noise_rule rule = {1ull << SV_OP_H, 0, &ch};
    sv_noise_model nm = {1, &rule, 0.0, 0.0};

    /* valid circuit, no arena yet: refused without touching the device */
    CHECK(sv_run_circuit(b, ops, 3, &nm, 7) == SV_ESTATE);
    /* qubit out of range */
    ops[1].q[1] = 4;
    CHECK(sv_run_circuit(b, ops, 3, &nm, 7) == SV_EINVAL);
    ops[1].q[1] = 3;
    /* repeated qubit in one op */
    ops[1].q[1] = 0;
    CHECK(sv_run_circuit(b, ops, 3, &nm, 7) == SV_EINVAL);
    ops[1].q[1] = 3;
    /* probabilities that do not sum to one */
    prob[0] = 0.5;
    CHECK(sv_run_circuit(b, ops, 3, &nm, 7) == SV_EINVAL);
    prob[0] = 0.97;
    /* readout probability outside [0, 1] */
    nm.readout_p01 = 1.5;
    CHECK(sv_run_circuit(b, ops, 3, &nm, 7) == SV_EINVAL);
    nm.readout_p01 = 0.0;
    /* results before any run */
    uint64_t mem[10];
    CHECK(sv_get_memory(b, mem, 10) == SV_ESTATE);
    CHECK(sv_batch_destroy(b) == SV_OK);
    printf("ok\n");
    return 0;
}
"""


@pytest.mark.skipif(shutil.which("gcc") is None, reason="no C compiler")
def test_c_program_builds_links_and_validates(tmp_path):
    if not os.path.exists(S.LIB_PATH):
        pytest.skip("library not built")
    src = tmp_path / "client.c"
    src.write_text(C_SOURCE)
    exe = tmp_path / "client"
    libdir = os.path.dirname(S.LIB_PATH)
    subprocess.check_call(["gcc", "-std=c99", "-Wall", "-Wextra", "-Werror", "-pedantic",
                           "-I", os.path.join(ROOT, "include"), str(src), "-o", str(exe),
                           "-L", libdir, "-lsvbatch", f"-Wl,-rpath,{libdir}"])
    out = subprocess.run([str(exe)], capture_output=True, text=True, timeout=120)
    assert out.returncode == 0, out.stdout + out.stderr
    assert out.stdout.strip().endswith("ok")
