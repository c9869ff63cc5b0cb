"""Scan of the library's own gfx950 machine code (CPU only; this file is
kept off GPU runs).  The kernels must never write through the scalar data
cache: no scalar stores, scalar atomics or scalar cache write-back."""
import os

from paper_1603_02526_amd import admm as A


def test_built_code_has_no_scalar_stores():
    """The library's own gfx950 code never writes through the scalar data
    cache (no scalar stores, scalar atomics or scalar cache write-back)."""
    import glob
    import shutil
    import subprocess
    import tempfile
    with tempfile.TemporaryDirectory() as td:
        so = os.path.join(td, "lib.so")
        shutil.copy(A.LIB_PATH, so)
        subprocess.run(["/opt/rocm/llvm/bin/llvm-objdump", "--offloading", so],
                       check=True, capture_output=True, cwd=td)
        cos = glob.glob(os.path.join(td, "lib.so.*gfx950*"))
        assert cos, "no gfx950 code object found in the library"
        found = []
        n_kernels = 0
        for co in cos:
            dis = subprocess.run(["/opt/rocm/llvm/bin/llvm-objdump", "-d", co],
                                 capture_output=True, text=True, check=True).stdout
            n_kernels += dis.count("s_endpgm")
            for line in dis.splitlines():
                ins = line.strip().split(" ")[0] if line.strip() else ""
                if ins.startswith(("s_store", "s_atomic", "s_buffer_store", "s_buffer_atomic",
                                   "s_dcache_wb", "s_scratch_store")):
                    found.append(line.strip())
        assert n_kernels > 10
        assert not found, found[:5]
