"""GPU test of jf_fidelity_noalloc, the entry point that allocates nothing: it runs a plan on the
library's static per-GPU scratch.  Each result is checked against jf_fidelity_alg1 / alg2 with a
caller workspace (the same kernels) at the parity bar of the form: |dF_J| and per-term |dt| within
1e-12 for complex128, |dF_J| within 1e-6 for complex64."""
import sys

import numpy as np
import pytest

from paper_2103_11595_amd import instances as gen
from paper_2103_11595_amd import jf

pytestmark = pytest.mark.gpu
TOL = {"c128": 1e-12, "c64": 1e-6}


def say(*a):
    print("[gpu-test]", *a, flush=True)
    sys.stdout.flush()


def _check_alg1(p, dtype, stream=None):
    ref = jf.jf_fidelity_alg1(p, stream=stream, want_terms=True)
    got = jf.jf_fidelity_noalloc(p, stream=stream, want_terms=True)
    assert abs(got["fj"] - ref["fj"]) <= TOL[dtype]
    assert abs(got["one_minus_fj"] - ref["one_minus_fj"]) <= TOL[dtype]
    assert got["kraus_terms"] == ref["kraus_terms"]
    if dtype == "c128":
        assert np.max(np.abs(got["terms"] - ref["terms"])) <= 1e-12
    return got


@pytest.mark.parametrize("dtype", ["c128", "c64"])
def test_noalloc_two_calls_second_smaller(dtype):
    import torch
    torch.cuda.set_device(0)
    big = jf.plan(gen.random_circuit(11, 250, 3, 1e-3, 1e-2, 25), 1, dtype)
    small = jf.plan(gen.random_circuit(9, 150, 2, 1e-3, 1e-2, 11), 1, dtype)
    assert big.info()["workspace_bytes"] > small.info()["workspace_bytes"]
    assert big.info()["workspace_bytes"] <= jf.JF_NOALLOC_BYTES
    assert big.info()["max_log2_intermediate"] > 11   # step kernels, tables in the scratch
    say("noalloc", dtype, "n=11 then n=9")
    a = _check_alg1(big, dtype)
    b = _check_alg1(small, dtype)
    # the scratch now holds the smaller plan's tables: the larger one copies its own in again
    say("noalloc", dtype, "n=11 again, then on a side stream")
    assert _check_alg1(big, dtype)["fj"] == a["fj"]
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        assert _check_alg1(small, dtype, stream=s)["fj"] == b["fj"]
    torch.cuda.synchronize()


def test_noalloc_algorithm_two_and_the_small_workload():
    import torch
    torch.cuda.set_device(0)
    p2 = jf.plan(gen.config5(), 2, "c64")          # 36-qubit chain, Algorithm II
    say("noalloc alg2 36-qubit chain c64")
    ref = jf.jf_fidelity_alg2(p2)
    got = jf.jf_fidelity_noalloc(p2)
    assert abs(got["fj"] - ref["fj"]) <= 1e-6 and abs(got["imag_residual"] - ref["imag_residual"]) <= 1e-6
    p1 = jf.plan(gen.config1(), 1, "c128")         # n=5 workload: the persistent LDS kernel
    say("noalloc n=5 workload c128")
    _check_alg1(p1, "c128")
    # traces exist for Algorithm I only: JF_E_ARG before anything is written
    r, buf = jf.jf_result(), (jf.C.c_double * 2)()
    assert jf.lib().jf_fidelity_noalloc(p2.ptr, None, jf.C.byref(r), buf) == -1


def test_noalloc_rejects_a_plan_beyond_the_scratch():
    p = jf.plan(gen.config2(), 1, "c64")           # n=16 workload: ~1 GiB of workspace
    assert p.info()["workspace_bytes"] > jf.JF_NOALLOC_BYTES
    say("noalloc rejects the n=16 plan")
    with pytest.raises(jf.JfError) as e:
        jf.jf_fidelity_noalloc(p)
    assert e.value.status == -6
    assert "no-allocation scratch" in str(e.value)
