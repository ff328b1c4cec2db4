"""Run the counter calibration probe (read_probe.hip): one read of a buffer of
known size with scalar loads, then one with vector loads, so that rocprofv3's
FETCH_SIZE for each can be compared with the bytes read, e.g.

    rocprofv3 --pmc FETCH_SIZE -d <dir> -- python3 tests/probes/read_probe.py --mib 1024

Compiles the probe with hipcc for gfx950 into a temporary directory first.
"""
import argparse
import ctypes
import os
import subprocess
import sys
import tempfile

HERE = os.path.dirname(os.path.abspath(__file__))


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--mib", type=int, default=1024)
    ap.add_argument("--blocks", type=int, default=4096)
    args = ap.parse_args()
    tmp = tempfile.mkdtemp()
    so = os.path.join(tmp, "libread_probe.so")
    subprocess.run(["hipcc", "-O3", "--offload-arch=gfx950", "-fPIC", "-shared", "-Xclang", "-target-feature",
                    "-Xclang", "-packed-fp32-ops", os.path.join(HERE, "read_probe.hip"), "-o", so], check=True)
    import torch
    bytes_ = args.mib << 20
    assert bytes_ % (64 * args.blocks) == 0
    src = torch.ones(bytes_ // 4, dtype=torch.int32, device="cuda")
    out = torch.empty(64 * args.blocks, dtype=torch.int32, device="cuda")
    torch.cuda.synchronize()
    lib = ctypes.CDLL(so)
    lib.read_probe.argtypes = [ctypes.c_int, ctypes.c_void_p, ctypes.c_uint64, ctypes.c_uint32, ctypes.c_void_p]
    lib.read_probe.restype = ctypes.c_int
    for kind, name in ((0, "scalar"), (1, "vector")):
        rc = lib.read_probe(kind, src.data_ptr(), bytes_, args.blocks, out.data_ptr())
        if rc != 0:
            print(f"read_probe {name} failed: {rc}", file=sys.stderr)
            return 1
        print(f"read_probe {name}: {bytes_} bytes read", flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
