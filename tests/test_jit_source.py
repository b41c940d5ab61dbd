"""The run-time compiled small-block kernel's source (held as a string in
the library) compiles for gfx950 with the library's compiler flags, for
FP64 and FP32 and for shapes with and without a k tail; CPU only."""
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")


def _source():
    txt = open(os.path.join(ROOT, "paper_1910_04796_amd", "csrc", "jit.hip")).read()
    m = re.search(r'R"JIT\((.*?)\)JIT"', txt, re.S)
    assert m, "kernel source string not found"
    return m.group(1)


@pytest.mark.parametrize("t,m,n,k", [("double", 23, 23, 23), ("float", 5, 32, 13), ("double", 64, 48, 64),
                                     ("double", 22, 22, 22), ("float", 16, 16, 3)])
def test_jit_source_compiles(tmp_path, t, m, n, k):
    if not os.path.exists(HIPCC):
        pytest.skip("hipcc not available")
    src = (_source().replace("@T@", t).replace("@F64@", "1" if t == "double" else "0")
           .replace("@M@", str(m)).replace("@N@", str(n)).replace("@K@", str(k)))
    f = tmp_path / "jit.hip"
    f.write_text('#include <hip/hip_runtime.h>\n' + src)
    r = subprocess.run([HIPCC, "--offload-arch=gfx950", "-O3", "-std=c++17", "-Xclang", "-target-feature",
                        "-Xclang", "-packed-fp32-ops", "--cuda-device-only", "-c", str(f), "-o",
                        str(tmp_path / "jit.o")], capture_output=True, text=True)
    assert r.returncode == 0, r.stderr[-2000:]
