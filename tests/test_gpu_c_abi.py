"""The C-ABI used from plain C, with no Python or torch in the process:
tests/c_abi_decode.c samples and decodes through libmcmcdec.so alone, and
its decisions equal those of the Python binding on the same seed."""

import os
import shutil
import subprocess
import sys

import numpy as np
import pytest

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

import paper_1302_2669_amd as mc  # noqa: E402

HERE = os.path.dirname(os.path.abspath(__file__))
PKG = os.path.join(os.path.dirname(HERE), "paper_1302_2669_amd")
ROCM = "/opt/rocm"


@pytest.fixture(scope="module")
def c_exe(tmp_path_factory):
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a HIP device")
    cc = shutil.which("gcc") or shutil.which("cc")
    if cc is None:
        pytest.skip("no C compiler on this machine")
    out = tmp_path_factory.mktemp("c_abi") / "c_abi_decode"
    # host-only C: the library brings every kernel
    subprocess.run([cc, "-std=c99", "-O2", "-D__HIP_PLATFORM_AMD__", f"-I{ROCM}/include",
                    os.path.join(HERE, "c_abi_decode.c"), "-o", str(out), f"-L{PKG}", "-lmcmcdec",
                    f"-L{ROCM}/lib", "-lamdhip64", f"-Wl,-rpath,{PKG}", f"-Wl,-rpath,{ROCM}/lib"],
                   check=True, capture_output=True)
    return str(out)


def test_c_program_matches_python_binding(c_exe, tmp_path):
    L, p, sweeps, chains, n, seed = 9, 0.12, 40, 2, 4096, 0x1302266900000099
    print(f"C-ABI program L={L} p={p} n={n}", flush=True)
    sys.stdout.flush()
    res = subprocess.run([c_exe, str(L), str(p), str(sweeps), str(chains), str(n), hex(seed),
                          str(tmp_path / "out.txt")], capture_output=True, text=True, timeout=120)
    assert res.returncode == 0, res.stderr
    assert res.stdout.startswith("ok ")
    got = np.loadtxt(tmp_path / "out.txt", dtype=np.int64).reshape(n, 2)
    syn, cls, _ = mc.sample_errors(L, p, seed, n, device="cuda")
    out = mc.decode_batch(syn, L, p, sweeps, seed, chains=chains, want_correction=False)
    torch.cuda.synchronize()
    assert np.array_equal(got[:, 1], cls.cpu().numpy().astype(np.int64))
    assert np.array_equal(got[:, 0], out["chosen"].cpu().numpy().astype(np.int64))
