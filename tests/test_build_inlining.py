"""The matrix-core kernels inline every device helper (CPU test: compiles
to gfx950 assembly only). A helper the compiler leaves as a call addresses
its LDS operands through flat pointers and its callers spill around the
call; the density-matrix kernel ran 526 instead of 380 ms per launch at
10x10 D=5 chi=25 when the eigensolver and the product routine were called
out of line. The build's flags (the AMDGPU inliner's basic-block budget
raised, the strip steps marked inline) keep every kernel of these files
free of calls; the canonical path's Jacobi helpers (env.hip and the files
that include it) are called on purpose and are not checked here."""
import os
import subprocess

import pytest

from paper_2503_12557_amd import build as B

FILES = ["env_dm.hip", "strip.hip"]


@pytest.mark.parametrize("src", FILES)
def test_no_out_of_line_calls(tmp_path, src):
    try:
        cc = B.hipcc()
    except RuntimeError:
        pytest.skip("hipcc not available")
    out = tmp_path / (src + ".s")
    cmd = [cc, *B.flags(), "--cuda-device-only", "-S", os.path.join(B.CSRC, src), "-o", str(out)]
    r = subprocess.run(cmd, capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-3000:]
    asm = out.read_text()
    assert "s_swappc_b64" not in asm, f"{src}: a device helper is called out of line"
