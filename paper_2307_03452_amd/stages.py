"""Per-stage breakdown of the fused (ab|cd) kernel, in the manner of the
paper's Table 2 (share of cycles and FLOP rate per sub-kernel), measured with
the stage-timer build of the library (liberi4_stages.so, built by
`python -m paper_2307_03452_amd.build --stage-timers`).

  python -m paper_2307_03452_amd.stages [--workloads iiii_k1 iiii_k5 gggg_k1] [--reps 2] [--out file.md]

Wave 0 of every workgroup reads the shader clock after each barrier that ends
a stage (pair data; Boys function and bra 1-d tables; the recursion of
eq. (md1); the first transform; the tile move and ket tables; the second
transform with the output write) and the sums over all workgroups are read
back.  Shares are of the summed workgroup cycles; a stage's FLOP rate is its
matrix FLOPs over its share of the launch's wall time.  The timer build adds a
clock read per stage, so its wall time is a little above the normal build's.
"""
import argparse
import ctypes
import os
import sys
import time

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HERE = os.path.dirname(os.path.abspath(__file__))
STAGES = ("pair data", "Boys + bra tables", "recursion [r]", "first transform", "tile move + ket tables",
          "second transform + write")
FP64_PEAK_TFLOPS = 78.6


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--workloads", nargs="*", default=["iiii_k1", "iiii_k5", "gggg_k1", "gggg_k3"],
                    help="bench.py workloads, or gggg_k3: (gg|gg) with 3 primitives per shell, 2048 quartets "
                         "(the contracted small classes that dominate the uneven batch)")
    ap.add_argument("--reps", type=int, default=2)
    ap.add_argument("--k5-quartets", type=int, default=64,
                    help="quartets of the K=5 batch to time (the first ones; all 512 take 2.6 s per call)")
    ap.add_argument("--out")
    a = ap.parse_args(argv)
    lib_path = os.path.join(HERE, "liberi4_stages.so")
    if not os.path.exists(lib_path):
        sys.exit(f"{lib_path} is missing: python -m paper_2307_03452_amd.build --stage-timers")
    os.environ["ERI4_LIBRARY"] = lib_path
    sys.path.insert(0, ROOT)
    import numpy as np
    import torch
    from paper_2307_03452_amd import eri4, inputs, metrics
    assert eri4.LIB_PATH == lib_path
    L = eri4.lib()
    L.eri4_stage_cycles.argtypes = [ctypes.c_void_p, ctypes.c_int]
    L.eri4_stage_cycles.restype = ctypes.c_int
    buf = np.zeros(7, dtype=np.uint64)

    def read(reset=True):
        assert L.eri4_stage_cycles(buf.ctypes.data_as(ctypes.c_void_p), int(reset)) == 0
        return buf.copy()

    sys.path.insert(0, ROOT)
    import bench
    eri4.init()
    lines = ["# Stage breakdown of the fused kernel (stage-timer build)", "",
             "Command: `python -m paper_2307_03452_amd.stages " + " ".join(argv or sys.argv[1:]) + "`", ""]
    extra = {"gggg_k3": dict(ls=(4, 4, 4, 4), K=3, nq=2048, seed=1011, exps=(0.05, 200.0),
                             desc="(gg|gg) l=4 Cartesian, K=3 per shell, 2048 quartets, exponents log-uniform "
                                  "[0.05,200], 8-Bohr cube")}
    for name in a.workloads:
        wl = extra[name] if name in extra else bench.WORKLOADS[name]
        b = bench.make_batch(wl)
        if name == "iiii_k5":
            b = inputs.subset(b, range(a.k5_quartets))
        d = lambda x: torch.from_numpy(np.ascontiguousarray(x)).cuda()
        C, E, Co, N = d(b.centers), d(b.exps), d(b.coefs), d(b.nprim)
        out = eri4.batch(wl["ls"], C, E, Co, N)
        torch.cuda.synchronize()
        read(True)
        t0 = time.perf_counter()
        for _ in range(a.reps):
            eri4.batch(wl["ls"], C, E, Co, N, out=out)
        torch.cuda.synchronize()
        wall = (time.perf_counter() - t0) / a.reps
        cyc = read(True).astype(np.float64)
        tiles = cyc[6] / a.reps
        tot = cyc[:6].sum()
        la, lb, lc, ld = wl["ls"]
        kb = wl["K"] * wl["K"]
        np_, nq_ = metrics.nherm(la + lb), metrics.nherm(lc + ld)
        nab, ncd = metrics.ncart(la) * metrics.ncart(lb), metrics.ncart(lc) * metrics.ncart(ld)
        f1 = b.nq * 2.0 * nab * (kb * np_) * (kb * nq_)
        f2 = b.nq * 2.0 * nab * (kb * nq_) * ncd
        flops = {3: f1, 5: f2}
        lines += [f"## {wl['desc']}" + (f" (first {b.nq} quartets)" if name == "iiii_k5" else ""), "",
                  f"{b.nq} quartets, {tiles:.0f} tiles per call, {wall * 1e3:.3f} ms per call (timer build); "
                  f"MD4 FLOPs {f1 + f2:.4g} -> {100 * (f1 + f2) / wall / 1e12 / FP64_PEAK_TFLOPS:.1f}% of FP64 peak", "",
                  "| stage | % of cycles | FLOP rate in its share of the time (% of FP64 peak) |", "|---|---|---|"]
        for i, st in enumerate(STAGES):
            share = cyc[i] / tot
            rate = ""
            if i in flops and share > 0:
                rate = f"{100 * flops[i] / (share * wall) / 1e12 / FP64_PEAK_TFLOPS:.1f}"
            lines.append(f"| {st} | {100 * share:.1f} | {rate} |")
        lines.append("")
        del out, C, E, Co, N
        torch.cuda.empty_cache()
    text = "\n".join(lines) + "\n"
    print(text, flush=True)
    if a.out:
        with open(a.out, "w") as f:
            f.write(text)


if __name__ == "__main__":
    main()
