"""The C ABI under host AddressSanitizer and UndefinedBehaviorSanitizer.

tests/abi_check.cpp is linked against a copy of the library whose host code
is instrumented (paper_1109_1205_amd.build.build_abi_check, run by
__graft_entry__.build(); device code is not instrumented).  It creates and
releases every kind of handle, takes the documented error returns, and runs
the ground state, H.v, propagation with the error estimate, the
allocation-free propagation and the four-step G in one call and step by
step on the half-filled 8-site ring (t = 1, U = 4, D = 4,900; a potential
0.3 on site 0 in H_ini).  The run must be free of sanitizer reports (leaks
included; the HIP and HSA runtimes' own allocations kept until exit are
suppressed by module) and its
numbers must match the oracle: E0 (Sec. 2), <0|H|0> = E0,
<0|e^{-iHt}|0> = e^{-iE0 t} at t = 0.5 (Sec. 3), and G^<, G^> on a 4 x 4
mesh (Sec. 4) to the G tolerance 1e-10."""
import dataclasses
import json
import os
import subprocess

import numpy as np
import pytest

import workloads as wl
from gpu_common import rel_err, say
from oracle import basis, greens, hamiltonian, lanczos

pytestmark = pytest.mark.gpu

BIN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "abi_check_asan")


def test_abi_under_host_sanitizers():
    assert os.path.exists(BIN), "sanitizer build missing: run __graft_entry__.build() first"
    supp = os.path.join(os.path.dirname(os.path.abspath(__file__)), "lsan_runtime.supp")
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:halt_on_error=1:abort_on_error=0",
               LSAN_OPTIONS=f"suppressions={supp}", UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    say("running the C ABI check under host ASan + UBSan")
    r = subprocess.run([BIN], capture_output=True, text=True, timeout=300, env=env)
    out = r.stdout + r.stderr
    assert "AddressSanitizer" not in out and "LeakSanitizer" not in out and "runtime error" not in out, out[-6000:]
    assert r.returncode == 0, out[-6000:]
    res = json.loads(r.stdout.strip().splitlines()[-1])

    H = wl.ring(8, 1.0, 4.0)
    eps = tuple(0.3 if i == 0 else 0.0 for i in range(8))
    Hi = dataclasses.replace(H, eps_up=eps, eps_dn=eps)
    sec = basis.Sector(8, 4, 4)
    v0 = np.cos(0.37 * np.arange(sec.dim)) + 0.1
    gs = lanczos.ground_state(hamiltonian.Hamiltonian(H, sec).apply, v0, tol=1e-13, max_iter=400)
    say("E0", res["E0"], gs.E0)
    assert abs(res["E0"] - gs.E0) <= 1e-12 * abs(gs.E0)
    assert abs(res["E0_from_Hv"] - gs.E0) <= 1e-11 * abs(gs.E0)
    assert 1.0 - 1e-10 <= res["fidelity2"] <= 1.0 + 1e-10
    ov = res["overlap_re"] + 1j * res["overlap_im"]
    assert abs(ov - np.exp(-1j * gs.E0 * 0.5)) < 1e-10
    assert 0.0 <= res["err_est"] < 1e-6

    ref = greens.four_step(Hi, H, 4, 4, [(0, 0), (0, 1)], 4, 0.1, 2, 15, v0, reorth="none")
    assert abs(res["E0_ini"] - ref["E0"]) <= 1e-12 * abs(ref["E0"])
    for key in ("G_lesser", "G_greater"):
        got = np.array([complex(a, b) for a, b in res[key]]).reshape(ref[key].shape)
        say(key, rel_err(got, ref[key]))
        assert rel_err(got, ref[key]) < 1e-10, key
