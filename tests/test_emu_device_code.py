"""The library's device code run on the CPU (tests/emu: the HIP sources
built for the host against an emulation of the device model, under
AddressSanitizer with every workspace allocation exactly its requested
size): small cases of assembly, both operators, both SpMM forms, both F w
product forms and a graph-replayed population agree with the oracle, and no
device access leaves its allocation (a sanitizer report aborts the child)."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_device_code_under_sanitizer(tmp_path):
    from tests.emu import build_emu, emu_ctx
    if not os.path.exists(build_emu.CLANG) or not os.path.exists(build_emu.asan_runtime()):
        pytest.skip("host clang with AddressSanitizer not available")
    lib = str(tmp_path / "libsdgp_emu.so")
    build_emu.build(os.path.join(ROOT, "paper_2205_09070_amd", "csrc"), lib)
    r = subprocess.run([sys.executable, "-u", os.path.join(ROOT, "tests", "emu", "replay.py"), lib, "ci"],
                       env=emu_ctx.emu_env(), capture_output=True, text=True, timeout=900, cwd=ROOT)
    print(r.stdout[-4000:])
    print(r.stderr[-6000:])
    assert r.returncode == 0, "emulated device code failed (see the sanitizer / emulator report above)"
    assert "results agree" in r.stdout
    shutil.rmtree(lib + ".src", ignore_errors=True)
