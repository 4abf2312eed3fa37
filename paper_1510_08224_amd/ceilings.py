"""Bandwidth ceilings of the GPU, the denominators beside the nominal
8 TB/s for the step kernel's roofline.

    python -m paper_1510_08224_amd.ceilings [--gib 2]

Streams of 2 GiB buffers (far beyond the 256 MB Infinity Cache): copy
(read + write), read-only, write-only, each over several grid sizes, and a
copy of one 16-byte element per thread; and the step's 14-plane pull
pattern without arithmetic on a 2048 x 2048 and a 4096 x 4096 lattice, in
separate planes and in the step kernel's row-interleaved layout.  Times
come from HIP events; one JSON object."""
from __future__ import annotations

import argparse
import ctypes
import json
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB = os.path.join(HERE, "libbwprobe.so")


def _lib():
    import torch  # noqa: F401  (one HIP runtime: torch's)
    if not os.path.exists(LIB):
        raise RuntimeError(f"{LIB} is missing: run `python -m paper_1510_08224_amd.build`")
    L = ctypes.CDLL(LIB)
    vp, ll = ctypes.c_void_p, ctypes.c_longlong
    L.bw_copy.argtypes = [vp, vp, ll, ctypes.c_int, vp]
    L.bw_read.argtypes = [vp, ll, ctypes.c_int, vp, vp]
    L.bw_write.argtypes = [vp, ll, ctypes.c_int, vp]
    L.bw_pull14.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, ll, vp]
    L.bw_copy1.argtypes = [vp, vp, ll, vp]
    L.bw_pull14_rows.argtypes = [ctypes.c_int, vp, vp, ctypes.c_int, ctypes.c_int, ctypes.c_int, vp]
    return L


def _time(fn, reps: int = 20) -> float:
    import torch
    for _ in range(3):
        assert fn() == 0
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        fn()
    e1.record()
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / 1e3 / reps


def measure(gib: float = 2.0) -> dict:
    import torch
    L = _lib()
    st = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    nb = int(gib * 2 ** 30)
    a = torch.zeros(nb // 4, dtype=torch.float32, device="cuda")
    b = torch.zeros_like(a)
    out = torch.zeros(1, dtype=torch.float32, device="cuda")
    pa, pb, po = ctypes.c_void_p(a.data_ptr()), ctypes.c_void_p(b.data_ptr()), ctypes.c_void_p(out.data_ptr())
    res = {"buffer_bytes": nb}
    for blocks in (1024, 2048, 4096, 16384):
        res[f"copy_blocks{blocks}_GBs"] = round(2 * nb / _time(lambda: L.bw_copy(pa, pb, nb, blocks, st)) / 1e9, 1)
        res[f"read_blocks{blocks}_GBs"] = round(nb / _time(lambda: L.bw_read(pa, nb, blocks, po, st)) / 1e9, 1)
        res[f"write_blocks{blocks}_GBs"] = round(nb / _time(lambda: L.bw_write(pb, nb, blocks, st)) / 1e9, 1)
    res["copy_1x16B_GBs"] = round(2 * nb / _time(lambda: L.bw_copy1(pa, pb, nb, st)) / 1e9, 1)
    res["copy_best_GBs"] = max(v for k, v in res.items() if k.startswith("copy_"))
    del a, b
    for n in (2048, 4096):
        for eb in (8, 4, 2):
            plane = n * n
            A = torch.zeros(14 * plane * eb // 4, dtype=torch.float32, device="cuda")
            B = torch.zeros_like(A)
            pA, pB = ctypes.c_void_p(A.data_ptr()), ctypes.c_void_p(B.data_ptr())
            t = _time(lambda: L.bw_pull14(eb, pA, pB, n, n, n, plane, st))
            res[f"pull14_n{n}_b{eb}_GBs"] = round(28 * eb * n * n / t / 1e9, 1)
            t = _time(lambda: L.bw_pull14_rows(eb, pA, pB, n, n, n, st))
            res[f"pull14_rows_n{n}_b{eb}_GBs"] = round(28 * eb * n * n / t / 1e9, 1)
            del A, B
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gib", type=float, default=2.0)
    args = ap.parse_args()
    import torch
    torch.cuda.set_device(0)
    print(json.dumps(measure(args.gib)), flush=True)


if __name__ == "__main__":
    main()
