"""Tuner of the persistent batched LU (stmg_batched_lu).

For each precision it times, on the GPU, factorizations of a seeded batch of
dense matrices with the sizes of the mixed Vanka patch batch (3D patches of
r in {1, 2, 3}, k in {0, 1, 2}: m = (k+1)(3(r+2)^3 + C(r+3, 3)), 85 ... 1185):

1. for every workgroup size (256 or 512 threads, the waves that factor one
   matrix), every workgroups-per-CU setting (which fixes the LDS budget of the
   launch) and every size class, the panel width (16, 8, 4) that factors a
   batch of that class alone fastest;
2. the whole mixed batch with each setting and its per-class widths;

and keeps the fastest setting.  The table is written to csrc/lu_tuning.h
(rebuild the library afterwards); the timings, with the one-launch-per-size-
class reference, are printed as one JSON line.

    python -m paper_2602_13841_amd.tune_lu [--batch 4096] [--reps 3] [--write] [--json F]
    python -m paper_2602_13841_amd.tune_lu --table-from F     # table from saved timings
"""
from __future__ import annotations

import argparse
import datetime
import json
import os
from math import comb

import numpy as np
import torch

from . import stmg

HERE = os.path.dirname(os.path.abspath(__file__))
CLASS_MAX = (128, 256, 512, 1024, 2048)
NBS = (16, 8, 4)
PRECS = (("f64", stmg.STMG_F64), ("f32", stmg.STMG_F32), ("f32_bf16", stmg.STMG_F32_BF16),
         ("f32_f16", stmg.STMG_F32_F16))


def patch_sizes(batch: int, seed: int = 6) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    r = rng.integers(1, 4, batch)
    k = rng.integers(0, 3, batch)
    return np.array([(kk + 1) * (3 * (rr + 2) ** 3 + comb(rr + 3, 3)) for rr, kk in zip(r, k)], dtype=np.int32)


def size_class(m: int) -> int:
    return next(c for c, mx in enumerate(CLASS_MAX) if m <= mx or c == len(CLASS_MAX) - 1)


class Batch:
    """Device copy of a batch of seeded matrices (entries U(-1, 1) plus a
    diagonal shift), restored before every timed factorization."""

    def __init__(self, sizes, dtype, seed=11):
        self.sizes = np.asarray(sizes, dtype=np.int32)
        m64 = self.sizes.astype(np.int64)
        self.a_off = np.concatenate([[0], np.cumsum(m64 * m64)[:-1]])
        self.p_off = np.concatenate([[0], np.cumsum(m64)[:-1]])
        total = int((m64 * m64).sum())
        g = torch.Generator(device="cuda")
        g.manual_seed(seed)
        self.orig = torch.rand(total, generator=g, device="cuda", dtype=dtype) * 2 - 1
        for i, m in enumerate(self.sizes):
            o = int(self.a_off[i])
            self.orig[o: o + int(m) * int(m): int(m) + 1] += 0.5 * float(m) ** 0.5
        self.A = torch.empty_like(self.orig)
        self.piv = torch.empty(int(m64.sum()), dtype=torch.int32, device="cuda")
        self.flops = float((2.0 / 3.0) * (m64.astype(float) ** 3).sum())

    def time(self, prec, config=None, reps=3):
        best = float("inf")
        for _ in range(reps):
            self.A.copy_(self.orig)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            stmg.batched_lu(self.A, self.a_off, self.sizes, self.piv, self.p_off, prec=prec, config=config)
            e1.record()
            torch.cuda.synchronize()
            best = min(best, e0.elapsed_time(e1) * 1e-3)
        return best


def tune(batch=4096, reps=3, log=print):
    sizes = patch_sizes(batch)
    result = {}
    for name, prec in PRECS:
        dt = torch.float64 if prec == stmg.STMG_F64 else torch.float32
        full = Batch(sizes, dt)
        classes = {}
        for c in range(len(CLASS_MAX)):
            sel = sizes[[size_class(int(m)) == c for m in sizes]]
            if len(sel):
                classes[c] = Batch(sel, dt)
        t_ref = full.time(prec, (0, None), reps)
        log(f"{name}: one launch per size class {t_ref * 1e3:.1f} ms ({full.flops / t_ref / 1e12:.2f} TFLOP/s)")
        best = None
        for threads in (256, 512):
            for wg in ((1, 2, 3, 4) if threads == 256 else (1, 2)):
                nb_best = []
                for c in range(len(CLASS_MAX)):
                    if c not in classes:
                        nb_best.append(16)
                        continue
                    ts = {nb: classes[c].time(prec, (wg, [nb] * len(CLASS_MAX), threads), reps) for nb in NBS}
                    nb_best.append(min(ts, key=ts.get))
                t = full.time(prec, (wg, nb_best, threads), reps)
                log(f"{name}: {threads} threads, {wg} workgroups per CU, panels {nb_best}: {t * 1e3:.1f} ms "
                    f"({full.flops / t / 1e12:.2f} TFLOP/s)")
                if best is None or t < best[0]:
                    best = (t, wg, nb_best, threads)
        result[name] = dict(wg_per_cu=best[1], threads=best[3], nb=best[2], seconds=best[0],
                            tflops=full.flops / best[0] / 1e12, per_class_launches_seconds=t_ref,
                            speedup=t_ref / best[0])
        del full, classes
        torch.cuda.empty_cache()
    props = torch.cuda.get_device_properties(0)
    result["device"] = f"{torch.cuda.get_device_name(0)} {getattr(props, 'gcnArchName', '')}".strip()
    result["date"] = datetime.date.today().isoformat()
    result["batch"] = batch
    return result


def write_table(result, path=os.path.join(HERE, "csrc", "lu_tuning.h")):
    dev = result.get("device", "")
    stamp = result.get("date", datetime.date.today().isoformat())
    rows = []
    for name, _ in PRECS:
        r = result[name]
        nb = ", ".join(str(v) for v in r["nb"])
        rows.append(f"    {{{r['wg_per_cu']}, {r['threads']}, {{{nb}}}}},   // {name}: {r['seconds'] * 1e3:.1f} ms, "
                    f"{r['tflops']:.2f} TFLOP/s; one launch per size class {r['per_class_launches_seconds'] * 1e3:.1f} ms")
    text = f"""// Launch parameters of the persistent batched LU (stmg_batched_lu), per
// precision: workgroups per CU (which sets the LDS budget of the launch) and
// the panel width per size class.  Written by paper_2602_13841_amd/tune_lu.py
// ({stamp}, {dev}) from the timings of the 4096-matrix mixed patch batch
// (sizes 85 ... 1185) noted beside each row.
#pragma once

namespace stmg {{

constexpr int LU_TUNE_CLASSES = 5;
constexpr int LU_CLASS_MAX[LU_TUNE_CLASSES] = {{128, 256, 512, 1024, 2048}};

struct LuTune {{
    int wg_per_cu;
    int threads;                 // per workgroup (one matrix): 256 or 512
    int nb[LU_TUNE_CLASSES];
}};

// index: 0 = FP64, 1 = FP32, 2 = FP32 with BF16 update operands, 3 = FP16
constexpr LuTune LU_TUNED[4] = {{
{chr(10).join(rows)}
}};

}} // namespace stmg
"""
    with open(path, "w") as f:
        f.write(text)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--batch", type=int, default=4096)
    ap.add_argument("--reps", type=int, default=3)
    ap.add_argument("--write", action="store_true", help="write csrc/lu_tuning.h")
    ap.add_argument("--json", help="also save the timings and the chosen table to this file")
    ap.add_argument("--table-from", help="write csrc/lu_tuning.h from a saved --json file (no GPU needed)")
    a = ap.parse_args()
    if a.table_from:
        with open(a.table_from) as f:
            write_table(json.load(f))
        return
    res = tune(a.batch, a.reps, log=lambda s: print(s, flush=True))
    if a.write:
        write_table(res)
    if a.json:
        with open(a.json, "w") as f:
            json.dump(res, f)
    print(json.dumps(res))


if __name__ == "__main__":
    main()
