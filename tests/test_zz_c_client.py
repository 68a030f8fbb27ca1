"""The C ABI used from a plain C++ program (tests/c_client/corr_client.cpp:
include/corr.h and the HIP runtime only, no Python in the process).  Its
int8 spectra must be the oracle's requantised real-input DFT (up to rounding
ties within the FP32 FFT error) and its visibilities the exact integer
correlation of those spectra; the error path it exercises must report
CORR_E_STATE."""
import os
import subprocess

import numpy as np
import pytest

import oracle
import paper_1305_5639_amd as corr
from helpers import fft_error_bound, say, tie_mismatches

pytestmark = pytest.mark.gpu
CLIENT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c_client", "corr_client")
N, C, A = 12, 64, 100


def test_c_client_matches_oracle(tmp_path):
    if not os.path.exists(CLIENT):
        pytest.skip("tests/c_client/corr_client is not built (tests/c_client/build.py)")
    say("C++ client of the C ABI")
    r = subprocess.run([CLIENT, str(tmp_path)], capture_output=True, text=True, timeout=120)
    say(r.stdout.strip() + r.stderr.strip())
    assert r.returncode == 0, r.stderr
    status = dict(l.split()[:2] for l in (tmp_path / "status.txt").read_text().splitlines())
    assert all(status[k] == "0" for k in ("corr_create", "corr_fengine_real8", "corr_xengine",
                                          "corr_dump_visibilities", "corr_copy_spectra", "corr_destroy"))
    assert status["corr_xengine_too_many"] == str(corr.CORR_E_STATE)
    x = np.fromfile(tmp_path / "samples.bin", np.int8).reshape(N, A * 2 * C)
    inv = np.fromfile(tmp_path / "inv.bin", np.float32)
    spec = np.fromfile(tmp_path / "spectra.bin", np.int8).reshape(A, C, N, 2)
    vis = np.fromfile(tmp_path / "vis.bin", np.int32).reshape(C, N * (N + 1) // 2, 2)
    S = np.swapaxes(spec, 1, 2)                                   # [A][N][C][2]
    assert np.array_equal(vis.astype(np.int64), oracle.xengine_i8(S))
    F = oracle.fengine_real8(x, C, A)                             # [A][N][C]
    q_ref = oracle.quantise(F, inv, "int8").astype(np.float64)
    y = F * inv.astype(np.float64)[None, None, :]
    eps = fft_error_bound(2 * C, np.sqrt(np.mean(np.abs(y) ** 2, axis=(0, 1))))[None, None, :, None] + 1e-30
    n_mis, n_bad = tie_mismatches(S.astype(np.float64), q_ref, np.stack([y.real, y.imag], -1), eps)
    say(f"  spectra: {n_mis} rounding-tie mismatches of {q_ref.size}, unexplained {n_bad}; "
        f"{int((np.abs(q_ref) == 127).sum())} values at the +-127 clamp")
    assert n_bad == 0 and n_mis <= max(2, q_ref.size // 100)
