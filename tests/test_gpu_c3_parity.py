"""The 20-qubit, 60-layer noisy workload (depolarizing 1e-3 / 1e-2,
amplitude damping 5e-3, readout 2%, 100,000 shots) against the FP64 oracle
on shot ids spread over the whole job, and the complex64 path against the
FP64 path.

The oracle's registers and decision margins for 256 ids come from
tests/golden/c3_oracle_registers.txt, written by
tests/golden/make_c3_oracle.py (it calls only the oracle)."""
import os

import numpy as np
import pytest

import workloads as W
from gpu_util import gpu_run, say

pytestmark = pytest.mark.gpu

HERE = os.path.dirname(os.path.abspath(__file__))
GOLDEN = os.path.join(HERE, "golden", "c3_oracle_registers.txt")
NEAR_TIE = 1e-9


def _golden():
    rows = [l.split() for l in open(GOLDEN) if l.strip() and not l.startswith("#")]
    ids = np.array([int(r[0]) for r in rows], dtype=np.int64)
    mem = np.array([int(r[1], 16) for r in rows], dtype=np.uint64)
    marg = np.array([float(r[2]) for r in rows], dtype=np.float64)
    return ids, mem, marg


def _blocks(ids):
    """Runs of consecutive ids: (first id, length)."""
    out, start = [], 0
    for i in range(1, len(ids) + 1):
        if i == len(ids) or ids[i] != ids[i - 1] + 1:
            out.append((int(ids[start]), i - start))
            start = i
    return out


@pytest.mark.parametrize("mode", ["batch", "branch"])
def test_c3_fp64_equals_oracle_on_ids_spread_over_the_job(mode):
    # complex128 storage, FP64 decisions: every sampled shot's register is
    # the oracle's (ids reached through shot_offset, up to 99,999). The
    # GPU's margins cover a subset of the oracle's decisions (draws below
    # the smallest eigenvalue of K_0^dagger K_0 need no state), so its
    # smallest margin per shot is never below the oracle's
    w = W.workload("c3_20q")
    ids, exp, exp_marg = _golden()
    got = np.zeros_like(exp)
    marg = np.zeros_like(exp_marg)
    ties = 0
    k = 0
    for first, length in _blocks(ids):
        say(f"case c3 c128 {mode}, shot ids {first}..{first + length - 1}")
        r = gpu_run(w["circuit"], w["noise"], length, dtype="c128", mode=mode, seed=w["seed"],
                    shot_offset=first, want_margins=True)
        got[k:k + length] = r["memory"]
        marg[k:k + length] = r["margins"]
        ties += r["stats"]["near_ties"]
        k += length
    bad = np.nonzero(got != exp)[0]
    say(f"{len(ids)} ids, mismatches {len(bad)}, oracle min margin {exp_marg.min():.3e} "
        f"({int(np.sum(exp_marg < NEAR_TIE))} shots below {NEAR_TIE:g}), GPU near-ties {ties}")
    for i in bad:
        say(f"  shot {ids[i]}: gpu {int(got[i]):x} oracle {int(exp[i]):x} "
            f"oracle margin {exp_marg[i]:.3e}")
    # a mismatch is allowed only as a near-tie: a decision whose oracle
    # margin is below 1e-9 (the two FP64 sums differ in rounding order)
    assert all(exp_marg[i] < NEAR_TIE for i in bad)
    assert len(bad) <= int(np.sum(exp_marg < NEAR_TIE))
    assert np.all(np.isfinite(marg))          # every shot samples its final state
    assert np.all(marg >= exp_marg * (1 - 1e-6) - 1e-13)
    assert ties == int(np.sum(marg < NEAR_TIE))


def test_c3_complex64_disagreements_are_adjacent_final_samples():
    # complex64 storage against complex128 on the same 10,000 shot ids with
    # readout error off, so the register is the sampled basis index. A
    # disagreement is either a final sample landing on the neighbouring
    # index (u*N falls between the complex64 and FP64 running sums of one
    # boundary of the 2^20-entry distribution) or a trajectory that went
    # another way at a Kraus choice (then the index is unrelated). The
    # second kind stays below 1e-3 of the shots; the output distributions
    # the final measurement samples from agree far closer than 1e-3
    w = W.workload("c3_20q")
    noise = dict(w["noise"], readout=[0.0, 0.0])
    shots = 10_000
    say(f"case c3 readout off, {shots} shots c64 and c128")
    a = gpu_run(w["circuit"], noise, shots, dtype="c64", seed=w["seed"])["memory"]
    b = gpu_run(w["circuit"], noise, shots, dtype="c128", seed=w["seed"])["memory"]
    diff = np.nonzero(a != b)[0]
    gap = np.abs(a[diff].astype(np.int64) - b[diff].astype(np.int64))
    adjacent = int(np.sum(gap == 1))
    other = len(diff) - adjacent
    say(f"disagreements {len(diff)} ({len(diff) / shots:.4%}), adjacent {adjacent}, "
        f"other {other} ({other / shots:.4%})")
    assert other / shots <= 1e-3
    assert len(diff) / shots <= 0.01
    for shot in (0, 4999, 9999):
        sa = gpu_run(w["circuit"], noise, 1, dtype="c64", seed=w["seed"], shot_offset=shot,
                     dump_shot=0)["state"]
        sb = gpu_run(w["circuit"], noise, 1, dtype="c128", seed=w["seed"], shot_offset=shot,
                     dump_shot=0)["state"]
        pa, pb = np.abs(sa) ** 2, np.abs(sb) ** 2
        tvd = 0.5 * np.sum(np.abs(pa / pa.sum() - pb / pb.sum()))
        say(f"shot {shot}: output-distribution TVD {tvd:.3e}, max amplitude error "
            f"{np.max(np.abs(sa - sb)):.3e}")
        assert tvd <= 1e-5
