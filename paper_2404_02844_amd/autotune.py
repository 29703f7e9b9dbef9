"""Offline tuner of the band kernels' workgroup shape (waves per workgroup, KS = 4 or 8).

Each band product runs one workgroup per 16-row tile; its KS waves split the tile's
contraction.  Eight waves give each tile twice the parallelism but halve each wave's
share of the contraction against the same reduction and epilogue, and they need twice
the LDS staging; which shape wins depends on the precision, the kernel, the number of
outcome columns (NT = Npad / 16) and the size, so it is measured.

For the batched / warm-start geometry family (D = round(1.2 M) probes with mu linearly
spaced to 1.1 M, band threshold 1e-16, lumped tail), M from 256 to 65536 and every
column-tile class, the tuner times the forward and the transposed product of each
precision with both shapes (HIP events around replayed launches on the problem's
stream) and writes pdt_tuning.h: per precision, kernel, column-tile class and size
class (log2 of the launch's workgroup count), KS = 8 where eight waves were faster by
more than 5 %, else 4.  Size classes outside the measured range take the nearest
measured class.

Usage (on the GPU):  python -m paper_2404_02844_amd.autotune --out <path to pdt_tuning.h>
"""
from __future__ import annotations

import argparse
import json
import sys
import time

import numpy as np

from . import _pdt

SIZES = (256, 512, 1024, 2048, 4096, 8192, 16384, 32768, 65536)
VARIANTS = ((0, _pdt.PDT_FP64), (1, _pdt.PDT_FP32), (2, _pdt.PDT_MIXED))
MARGIN = 1.05


def time_kernel(pb, kern: int, precision: int, reps: int) -> float:
    import torch
    stream = torch.cuda.current_stream()
    _pdt.pdt_replay_kernel(pb.handle, kern, precision, 3)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    _pdt.pdt_replay_kernel(pb.handle, kern, precision, reps)
    e1.record(stream)
    e1.synchronize()
    return e0.elapsed_time(e1) / reps * 1e-3


def measure(sizes=SIZES, nts=range(1, 13), reps: int = 20, log=print):
    """rows of (variant, kernel, nt, M, n_tiles, t_ks4, t_ks8)"""
    import torch
    rows = []
    for M in sizes:
        D = int(round(1.2 * M))
        mu = np.linspace(0.0, 1.1 * M, D)
        for nt in nts:
            N = 16 * nt
            P = np.full((D, N), 1.0 / N)
            pb = _pdt.Problem(mu, P, M, 1e-4, 1e-16, _pdt.PDT_TAIL_LUMP)
            n_tiles = ((D + 15) // 16, (M + 15) // 16)  # forward, transposed
            for var, prec in VARIANTS:
                X = torch.zeros((M, N), dtype=torch.float64, device="cuda")
                pb.solve(X, precision=prec, max_iters=3)
                t = {}
                for ks in (4, 8):
                    pb.set_tiles(prec, ks, ks)
                    for kernel, kern_id in ((0, 1), (1, 0)):  # forward = replay kernel 1, transposed = 0
                        t[(kernel, ks)] = time_kernel(pb, kern_id, prec, reps)
                pb.set_tiles(prec, 0, 0)
                for kernel in (0, 1):
                    rows.append((var, kernel, nt, M, n_tiles[kernel], t[(kernel, 4)], t[(kernel, 8)]))
            pb.close()
            log(f"[autotune] M={M} NT={nt} done")
    return rows


def size_class(n_tiles: int) -> int:
    """floor(log2(workgroups)), clamped to 0..15 (the same rule as choose_ks)."""
    return min(15, max(0, int(n_tiles).bit_length() - 1))


def decide(rows):
    """kKs[var][kernel][nt][class]: 8 where eight waves beat four by more than the margin."""
    table = [[[[4] * 16 for _ in range(13)] for _ in range(2)] for _ in range(3)]
    for var in range(3):
        for kernel in range(2):
            for nt in range(1, 13):
                pts = [(size_class(r[4]), r[5], r[6]) for r in rows if r[0] == var and r[1] == kernel and r[2] == nt]
                if not pts:
                    continue
                measured = {}
                for c, t4, t8 in pts:
                    measured.setdefault(c, []).append(8 if t8 * MARGIN < t4 else 4)
                got = {c: (8 if v.count(8) > v.count(4) else 4) for c, v in measured.items()}
                cs = sorted(got)
                for c in range(16):
                    near = min(cs, key=lambda m: (abs(m - c), m))
                    table[var][kernel][nt][c] = got[near]
    return table


def header(table) -> str:
    def row(v):
        return "{" + ", ".join(str(x) for x in v) + "}"
    blocks = []
    for v in range(3):
        kern = []
        for k in range(2):
            kern.append("{" + ", ".join(row(table[v][k][nt]) for nt in range(13)) + "}")
        blocks.append("    {" + ",\n     ".join(kern) + "}")
    body = ",\n".join(blocks)
    return f"""// Waves per workgroup (KS, 4 or 8) of the band kernels per precision, kernel, column-tile
// class NT and size class (floor(log2) of the launch's workgroup count, 0..15).
// Written by paper_2404_02844_amd/autotune.py from kernel timings on MI355X (gfx950):
// 8 where eight waves were measured faster than four by more than 5 %.
#pragma once

namespace pdt {{

// [variant: FP64, FP32, mixed][kernel: forward, transposed][NT = 0..12][size class]
constexpr unsigned char kKs[3][2][13][16] = {{
{body},
}};

inline int choose_ks(int variant, int kernel, int nt, long long n_tiles) {{
  if (variant < 0 || variant > 2 || kernel < 0 || kernel > 1 || nt < 1 || nt > 12) return 4;
  int c = 0;
  while (c < 15 && (n_tiles >> (c + 1)) > 0) ++c;
  return kKs[variant][kernel][nt][c] == 8 ? 8 : 4;
}}

}}  // namespace pdt
"""


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--out", default="")
    ap.add_argument("--raw", default="", help="also write the timings as JSON")
    ap.add_argument("--reps", type=int, default=20)
    args = ap.parse_args(argv)
    t0 = time.time()
    rows = measure(reps=args.reps, log=lambda *a: print(*a, flush=True))
    table = decide(rows)
    text = header(table)
    print(text, flush=True)
    print(f"[autotune] {len(rows)} timings in {time.time() - t0:.1f} s", flush=True)
    if args.out:
        with open(args.out, "w") as fh:
            fh.write(text)
    if args.raw:
        with open(args.raw, "w") as fh:
            json.dump([list(r) for r in rows], fh)


if __name__ == "__main__":
    sys.exit(main())
