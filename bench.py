"""Throughput of the batched exact Mallows-distance path on one MI355X.

Default (configuration 2): one step = one d2_assign over the whole workload
-- every object against every centroid (one transportation LP each, FP64
simplex) reduced to the nearest centroid (Alg. 2, Step 2 of the paper):
100,000 distributions (d=8, supports 1..16, 20-component Gaussian mixture,
Dirichlet(0.5) weights, FP32 storage) against 512 centroids of support 16,
51.2M LPs per step.  Inputs are resident in HBM before the timed region.
Prints one JSON line.

The default run also checks every row of configuration 2 against the
oracle (the oracle's time over all of them is the CPU baseline), and adds a
short serving leg of configuration 5 (Poisson queries against 1,024 resident
centroids: p50/p99 latency at 10k queries/s, the served capacity under
overload, parity of served results, and the plain per-pair solver on the
same queries).

Other workloads: --config 1 (200 x 10, d=3), --config 3 (50,000 x 256,
d=128), --config 4 (one segment's pairwise matrix, 4,096 objects, d=16,
8.4M pairs); --config 5 runs the serving loop (see paper_1302_0435_amd.serve).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

FP64_VECTOR_PEAK_TFLOPS = 78.6   # 256 CU x 4 SIMD x 16 lanes x 2 (FMA) x 2.4 GHz
HBM_PEAK_GBS = 8000.0
# Committed rocprofv3 summaries of each workload's dominant kernel, keyed by
# (configuration, cost mode).  The BF16 mode's MFMA cost tiles are computed
# inside its labelling kernel.
PROFILES = {
    (2, "f64"): "k_assign_cls0_f32_c2_100k_x512.txt",
    (3, "f64"): "k_assign_cls1_f32_c3_50k_x256_d128.txt",
    (3, "bf16"): "k_assign_bf16_f32_c3_50k_x256_d128.txt",
    (4, "f64"): "k_pairwise_q_cls2_f64_c4_4096.txt",
}
# the centroid update's dominant kernel (--op update), keyed by configuration
UPDATE_PROFILES = {2: "k_upd_solve_cls0_f32_c2_100k_x512.txt"}
# the given-cost LP kernel (--op cost), configuration 2 shapes
COST_PROFILES = {2: "k_emd_cost_cls0_c2_shapes_2m.txt"}
# the labelling kernel of the two-type distance of Eq. (9) (--op multi),
# which also writes each type's D^2 matrix
MULTI_PROFILES = {2: "k_assign_cls0_f32_c2_multi_type_all.txt"}
# the workgroup simplex on supports beyond 64 (--op large)
LARGE_PROFILES = {2: "k_emd_wg_f64_large_96_192.txt"}
# the hierarchy's dominant kernel (--op hierarchy): the free-weight centroid
# update of Step 2 (its labelling kernel has a summary of its own,
# k_assign_seg_cls0_f64_c2_hierarchy_100k.txt)
HIER_PROFILES = {2: "k_free_solve_f64_c2_hierarchy_100k.txt"}
KERNEL_SRCS = [os.path.join(ROOT, "paper_1302_0435_amd", "csrc", f)
               for f in ("d2_solver.h", "d2_shapes.h", "d2_kernels.hip")]
UPDATE_SRCS = [os.path.join(ROOT, "paper_1302_0435_amd", "csrc", f)
               for f in ("d2_solver.h", "d2_shapes.h", "d2_update.hip")]
COST_SRCS = [os.path.join(ROOT, "paper_1302_0435_amd", "csrc", f)
             for f in ("d2_solver.h", "d2_shapes.h", "d2_cost.hip")]
SEG_SRCS = [os.path.join(ROOT, "paper_1302_0435_amd", "csrc", f)
            for f in ("d2_solver.h", "d2_shapes.h", "d2_seg.hip")]
WG_SRCS = [os.path.join(ROOT, "paper_1302_0435_amd", "csrc", "d2_wg.hip")]


def kernel_sha(srcs=None) -> str:
    """Hash of the kernel sources with comments and blank space removed, so
    that a profile stays valid across edits that change no code."""
    import hashlib
    import re
    h = hashlib.sha256()
    for f in (srcs or KERNEL_SRCS):
        text = open(f, encoding="utf-8").read()
        text = re.sub(r"/\*.*?\*/", " ", text, flags=re.S)
        text = re.sub(r"//[^\n]*", " ", text)
        h.update(" ".join(text.split()).encode())
    return h.hexdigest()[:16]


def _read_profile(name):
    kv = {}
    try:
        with open(os.path.join(ROOT, "profiles", name)) as f:
            first = f.readline()
            for line in [first] + f.readlines():
                body = line.split("#", 1)[0].strip()
                if "=" in body:
                    for part in body.split():
                        if "=" in part:
                            k, v = part.split("=", 1)
                            kv[k] = v
        kv["_kernel"] = first.lstrip("# ").strip()
    except OSError:
        return None
    return kv


def profile_counters(cfg: int, cost: str, op: str = "assign"):
    """Counter figures of the dominant kernel from the committed rocprofv3
    summary, valid only while the kernel sources are unchanged."""
    if op == "update":
        kv = _read_profile(UPDATE_PROFILES.get(cfg, ""))
        sha = kernel_sha(UPDATE_SRCS)
    elif op == "cost":
        kv = _read_profile(COST_PROFILES.get(cfg, ""))
        sha = kernel_sha(COST_SRCS)
    elif op == "hierarchy":
        kv = _read_profile(HIER_PROFILES.get(cfg, ""))
        sha = kernel_sha(UPDATE_SRCS)
    elif op == "multi":
        kv = _read_profile(MULTI_PROFILES.get(cfg, ""))
        sha = kernel_sha()
    elif op == "large":
        kv = _read_profile(LARGE_PROFILES.get(cfg, ""))
        sha = kernel_sha(WG_SRCS)
    elif op != "assign":
        return None   # no committed profile of this workload
    else:
        kv = _read_profile(PROFILES.get((cfg, cost), ""))
        sha = kernel_sha()
    if not kv or kv.get("kernel_source_sha256_16") != sha:
        return None
    out = {"kernel": kv["_kernel"],
           "traffic": float(kv["hbm_bytes_per_dispatch"]),
           "valu_issue_busy": float(kv["valu_issue_busy_fraction"]),
           "lds_util_percent": float(kv["lds_util_percent"]),
           "profile_avg_ms": float(kv["avg_duration_ns"]) / 1e6}
    return out


def _cpu_model() -> str:
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def copy_calibration(mib: int) -> int:
    """A plain copy of known size: FETCH_SIZE / WRITE_SIZE of this kernel give
    the scale between the counters and true HBM bytes."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda:0")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4,
                      "launches": 3}), flush=True)
    return 0


# ------------------------------------------------------------- workloads


def _timed(fn, reps=2):
    """Mean seconds of fn() over reps calls after one warm call (device-synchronised)."""
    import torch
    fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        fn()
    torch.cuda.synchronize()
    return (time.perf_counter() - t0) / reps


def _pinned_set(S):
    import torch
    return [torch.from_numpy(np.ascontiguousarray(a)).pin_memory() for a in (S.offsets, S.points, S.weights)]


def _h2d(d2, host, dev_bufs, max_support):
    for h, d in zip(host, dev_bufs):
        d.copy_(h, non_blocking=True)
    return d2.DeviceSet(dev_bufs[0], dev_bufs[1], dev_bufs[2], max_support)


class AssignWorkload:
    """d2_assign of a configuration's objects against its centroids."""

    def __init__(self, cfg, d2, dev, init, schedule, n=None, cost_mode=0):
        import synth
        self.cfg = cfg
        self.cost_mode = cost_mode
        self.spec = synth.CONFIGS[cfg]
        self.X = synth.make_data(cfg, n=n)
        self.Z = synth.make_centroids(cfg)
        self.d2 = d2
        self.h = d2.Handle(0)
        self.Xd = d2.DeviceSet.from_ragged(self.X, dev)
        self.Zd = d2.DeviceSet.from_ragged(self.Z, dev)
        self.opts = d2.Opts(init=init, schedule=schedule, cost_mode=cost_mode)
        self.pairs = self.X.n * self.Z.n
        self.out = None

    def step(self):
        self.out = self.d2.d2_assign(self.h, self.Xd, self.Zd, self.opts)

    def flops(self):
        """Pivot-free work: per pair the ground-cost tile (3 t s d: difference,
        square, add) plus one certifying pricing pass (3 t s)."""
        ts = np.diff(self.X.offsets).astype(np.float64)
        ss = np.diff(self.Z.offsets).astype(np.float64)
        return float(ts.sum() * ss.sum() * (3 * self.X.points.shape[1] + 3))

    def bytes(self):
        X, Z = self.X, self.Z
        return float(X.points.nbytes + X.weights.nbytes + X.offsets.nbytes + Z.points.nbytes +
                     Z.weights.nbytes + Z.offsets.nbytes + X.n * (4 + 8))

    def failed(self):
        return int((self.out[3].cpu().numpy() != 0).sum())

    def plain_baseline(self, rows=2000):
        """The plain per-pair solver (one wavefront per pair in input order,
        north-west corner, FP64 cost, no binning, no graph) on the first rows."""
        d2 = self.d2
        sub = self.X.subset(np.arange(min(rows, self.X.n)))
        Xs = d2.DeviceSet.from_ragged(sub, "cuda:0")
        opts = d2.Opts(init=d2.D2_INIT_NWC, schedule=d2.D2_SCHED_PLAIN, flags=d2.D2_FLAG_EAGER)
        dt = _timed(lambda: d2.d2_assign(self.h, Xs, self.Zd, opts))
        return {"value": sub.n * self.Z.n / dt, "unit": "distances/s",
                "sample": f"first {sub.n} objects x all {self.Z.n} centroids"}

    def end_to_end(self):
        """One step with the objects copied in from pinned host memory and
        labels and minima copied back (the centroids stay resident)."""
        import torch
        d2 = self.d2
        host = _pinned_set(self.X)
        bufs = [torch.empty_like(hh, device="cuda:0") for hh in host]
        lab_h = torch.empty(self.X.n, dtype=torch.int32).pin_memory()
        best_h = torch.empty(self.X.n, dtype=torch.float64).pin_memory()

        def run():
            Xd = _h2d(d2, host, bufs, self.Xd.max_support)
            lab, best, _, _ = d2.d2_assign(self.h, Xd, self.Zd, self.opts)
            lab_h.copy_(lab, non_blocking=True)
            best_h.copy_(best, non_blocking=True)
        dt = _timed(run)
        return {"ms_per_step": dt * 1e3, "value": self.pairs / dt,
                "input_bytes": int(sum(hh.numel() * hh.element_size() for hh in host))}

    def config(self):
        s = self.spec
        return {"workload": s["name"], "n": self.X.n, "k": self.Z.n, "d": self.X.points.shape[1],
                "t_range": list(s["t_range"]), "s": s["s"], "inputs": s["dtype"],
                "pairs_per_step": self.pairs}

    def cpu_baseline(self, target_s, init_oracle, all_rows=False):
        """The oracle timed on this host's cores on a bounded sample of rows
        (all centroids per row), or on every row with ``all_rows``; also checks
        the device results for those rows."""
        import oracle
        import synth
        from tests.parity import coupling_cost
        X, Z = self.X, self.Z
        g_labels = self.out[0].cpu().numpy()
        g_best = self.out[1].cpu().numpy()
        threads = oracle.default_threads()
        if all_rows:
            rows = np.arange(X.n)
        else:
            rows = synth.sample_rows(self.cfg, X.n, min(64, X.n), tag=1)
            t0 = time.perf_counter()
            oracle.assign(X.subset(rows), Z, init=init_oracle, threads=threads, want_all=False)
            rate = len(rows) * Z.n / max(time.perf_counter() - t0, 1e-6)
            n_rows = int(min(X.n, max(16, target_s * rate / Z.n)))
            rows = synth.sample_rows(self.cfg, X.n, n_rows, tag=2)
        sub = X.subset(rows) if not all_rows else X
        t0 = time.perf_counter()
        o_lab, o_best, _, o_st, _ = oracle.assign(sub, Z, init=init_oracle, threads=threads,
                                                  want_all=False)
        dt = time.perf_counter() - t0
        base = {"value": len(rows) * Z.n / dt, "unit": "distances/s", "cores": threads,
                "kind": "oracle",
                "sample": f"{'all' if all_rows else 'seeded'} {len(rows)} rows x all {Z.n} centroids "
                          f"({len(rows) * Z.n} LPs), {dt:.1f} s, "
                          f"{'Vogel' if init_oracle else 'north-west-corner'} start",
                "cpu_model": _cpu_model()}
        if self.cost_mode == 1:
            # BF16 ground cost: report its error against the FP64 oracle
            gb = g_best[rows]
            rel = np.abs(gb - o_best) / np.maximum(np.abs(o_best), 1e-300)
            base["bf16_vs_fp64"] = {
                "rows": len(rows), "label_agreement": float(np.mean(g_labels[rows] == o_lab)),
                "best_rel_err_max": float(rel.max()), "best_rel_err_median": float(np.median(rel))}
            return base
        fails = 0
        for k, i in enumerate(rows):
            ob, gb = o_best[k], g_best[i]
            if o_lab[k] == g_labels[i] and abs(gb - ob) <= 1e-10 * abs(ob):
                continue
            floor = 1e-14 * coupling_cost(*sub.bag(k), *Z.bag(int(o_lab[k])))
            if abs(gb - ob) > max(1e-10 * abs(ob), floor):
                fails += 1
        base.update({"parity_checked": len(rows), "parity_failures": fails})
        return base


class PairwiseWorkload:
    """d2_pairwise over one segment (configuration 4)."""

    def __init__(self, cfg, d2, dev, init, schedule, n=None, tune=False):
        import synth
        self.cfg = cfg
        self.spec = synth.CONFIGS[cfg]
        self.X = synth.make_data(cfg, n=n)
        self.d2 = d2
        self.h = d2.Handle(0)
        self.Xd = d2.DeviceSet.from_ragged(self.X, dev)
        self.opts = d2.Opts(init=init, schedule=schedule)
        self.pairs = self.X.n * (self.X.n - 1) // 2
        self.tuned_ms = None
        if tune and schedule == d2.D2_SCHED_AUTO:
            _, _, self.tuned_ms = d2.d2_tune_pairwise(self.h, self.Xd, self.opts)
        self.out = None

    def step(self):
        self.out = self.d2.d2_pairwise(self.h, self.Xd, self.opts)

    def flops(self):
        ts = np.diff(self.X.offsets).astype(np.float64)
        return float((ts.sum() ** 2 - (ts ** 2).sum()) / 2 * (3 * self.X.points.shape[1] + 3))

    def bytes(self):
        X = self.X
        return float(X.points.nbytes + X.weights.nbytes + X.offsets.nbytes + self.pairs * 8)

    def failed(self):
        return int((self.out[1].cpu().numpy() != 0).sum())

    def plain_baseline(self, objects=1024):
        d2 = self.d2
        sub = self.X.subset(np.arange(min(objects, self.X.n)))
        Xs = d2.DeviceSet.from_ragged(sub, "cuda:0")
        opts = d2.Opts(init=d2.D2_INIT_NWC, schedule=d2.D2_SCHED_PLAIN, flags=d2.D2_FLAG_EAGER)
        dt = _timed(lambda: d2.d2_pairwise(self.h, Xs, opts))
        return {"value": sub.n * (sub.n - 1) / 2 / dt, "unit": "distances/s",
                "sample": f"all pairs of the first {sub.n} objects"}

    def end_to_end(self):
        import torch
        d2 = self.d2
        host = _pinned_set(self.X)
        bufs = [torch.empty_like(hh, device="cuda:0") for hh in host]
        out_h = torch.empty(self.pairs, dtype=torch.float64).pin_memory()

        def run():
            Xd = _h2d(d2, host, bufs, self.Xd.max_support)
            out, _ = d2.d2_pairwise(self.h, Xd, self.opts)
            out_h.copy_(out, non_blocking=True)
        dt = _timed(run)
        return {"ms_per_step": dt * 1e3, "value": self.pairs / dt,
                "input_bytes": int(sum(hh.numel() * hh.element_size() for hh in host)),
                "output_bytes": self.pairs * 8}

    def config(self):
        s = self.spec
        return {"workload": s["name"], "n": self.X.n, "d": self.X.points.shape[1],
                "t_range": list(s["t_range"]), "single_atom": s["single_atom"],
                "inputs": s["dtype"], "pairs_per_step": self.pairs,
                "autotuned_ms": self.tuned_ms}

    def cpu_baseline(self, target_s, init_oracle, all_pairs=False):
        """The oracle on a seeded sample of pairs i < j sized to ``target_s``,
        or on every pair with ``all_pairs``; checks the device's values there."""
        import oracle
        import synth
        from tests.parity import pair_tolerance_fast
        X = self.X
        g = self.out[0].cpu().numpy()
        threads = oracle.default_threads()
        n = X.n

        def sample(count, tag):
            p = synth.sample_pairs(self.cfg, n, n, count * 3, tag=tag)
            return p[p[:, 0] < p[:, 1]][:count]
        if all_pairs:
            iu = np.triu_indices(n, 1)
            p = np.stack(iu, 1).astype(np.int64)          # squareform order
        else:
            p = sample(2000, 1)
            t0 = time.perf_counter()
            oracle.emd_batch(X, X, p, init=init_oracle, threads=threads)
            rate = len(p) / max(time.perf_counter() - t0, 1e-6)
            p = sample(int(max(1000, target_s * rate)), 2)
        t0 = time.perf_counter()
        o, o_st, _ = oracle.emd_batch(X, X, p, init=init_oracle, threads=threads)
        dt = time.perf_counter() - t0
        idx = p[:, 0] * n - p[:, 0] * (p[:, 0] + 1) // 2 + (p[:, 1] - p[:, 0] - 1)
        tol = np.maximum(1e-10 * np.abs(o), pair_tolerance_fast(X, X, p))
        fails = int((~(np.abs(g[idx] - o) <= tol)).sum()) + int((o_st != 0).sum())
        return {"value": len(p) / dt, "unit": "distances/s", "cores": threads, "kind": "oracle",
                "sample": f"{'all' if all_pairs else 'seeded'} {len(p)} pairs i<j, {dt:.1f} s, "
                          f"{'Vogel' if init_oracle else 'north-west-corner'} start",
                "parity_checked": len(p), "parity_failures": fails, "cpu_model": _cpu_model()}


class UpdateWorkload:
    """d2_centroid_update: one pass of the constrained D2 centroid update
    (Alg. 2 Step 3*) over a configuration's objects, each against its own
    centroid (centroid weights uniform, 1/s).  The labels are the nearest
    centroids, from one d2_assign in the untimed set-up."""

    metric = "constrained D2 centroid update: objects/sec (member LP + Eq. (2) mean + objective)"
    unit = "objects/s"

    def __init__(self, cfg, d2, dev, init, schedule, n=None):
        import synth
        import torch
        self.cfg = cfg
        self.spec = synth.CONFIGS[cfg]
        self.X = synth.make_data(cfg, n=n)
        Z = synth.make_centroids(cfg)
        w = np.concatenate([np.full(int(t), 1.0 / int(t)) for t in np.diff(Z.offsets)])
        self.Z = synth.RaggedSet(Z.offsets, Z.points, w.astype(Z.points.dtype))
        self.d2 = d2
        self.h = d2.Handle(0)
        self.Xd = d2.DeviceSet.from_ragged(self.X, dev)
        self.Zd = d2.DeviceSet.from_ragged(self.Z, dev)
        self.opts = d2.Opts(init=init, schedule=schedule)
        self.labels = d2.d2_assign(self.h, self.Xd, self.Zd, d2.Opts(init=init))[0]
        torch.cuda.synchronize()
        self.pairs = self.X.n
        self.out = None

    def step(self):
        self.out = self.d2.d2_centroid_update(self.h, self.Xd, self.Zd, self.labels, self.opts)

    def flops(self):
        """Pivot-free work of the member problems: per member the ground-cost
        tile (3 t s d) plus one certifying pricing pass (3 t s)."""
        lab = self.labels.cpu().numpy()
        ts = np.diff(self.X.offsets).astype(np.float64)
        ss = np.diff(self.Z.offsets).astype(np.float64)[lab]
        return float((ts * ss).sum() * (3 * self.X.points.shape[1] + 3))

    def bytes(self):
        X, Z = self.X, self.Z
        return float(X.points.nbytes + X.weights.nbytes + X.offsets.nbytes + 2 * Z.points.nbytes +
                     Z.weights.nbytes + Z.offsets.nbytes + X.n * (4 + 4) + Z.n * 20)

    def failed(self):
        return int((self.out[4].cpu().numpy() != 0).sum())

    def config(self):
        s = self.spec
        return {"workload": s["name"] + " centroid update", "n": self.X.n, "k": self.Z.n,
                "d": self.X.points.shape[1], "t_range": list(s["t_range"]), "s": s["s"],
                "inputs": s["dtype"], "centroid_weights": "uniform", "objects_per_step": self.X.n}

    def cpu_baseline(self, target_s, init_oracle):
        """The oracle's centroid update on the members of a seeded sample of
        clusters; also checks the device's moved atoms and objectives there."""
        import oracle
        import synth
        X, Z = self.X, self.Z
        lab = self.labels.cpu().numpy()
        z, e1, e3 = (t.cpu().numpy() for t in self.out[:3])
        order = synth.rng_for(self.cfg, synth.STREAM_SAMPLE, 300).permutation(Z.n)

        def run(k):
            pick = order[:k]
            rows = np.flatnonzero(np.isin(lab, pick))
            sub = X.subset(rows)
            t0 = time.perf_counter()
            res = oracle.centroid_update(sub, Z, lab[rows], init=init_oracle)
            return pick, rows, res, time.perf_counter() - t0

        _, rows, _, dt = run(2)
        per_obj = dt / max(len(rows), 1)
        k = int(min(Z.n, max(2, target_s / max(per_obj, 1e-9) / max(X.n / Z.n, 1))))
        pick, rows, (oz, oe1, oe3, ost), dt = run(k)
        fails = 0
        M = float(np.abs(X.points).max())
        for j in pick:
            a0, a1 = int(Z.offsets[j]), int(Z.offsets[j + 1])
            if np.abs(z[a0:a1] - oz[a0:a1]).max() > 1e-10 * M:
                fails += 1
            elif abs(e3[j] - oe3[j]) > 1e-10 * abs(oe3[j]) + 1e-14 * abs(oe1[j]):
                fails += 1
        return {"value": len(rows) / dt, "unit": "objects/s", "cores": 1, "kind": "oracle",
                "sample": f"members of {len(pick)} seeded clusters ({len(rows)} objects), "
                          f"{dt:.1f} s, {'Vogel' if init_oracle else 'north-west-corner'} start",
                "cpu_model": _cpu_model(), "parity_checked_clusters": len(pick),
                "parity_failures": fails}


class CostWorkload:
    """d2_emd_cost_batch: transport LPs over caller-given FP64 cost matrices,
    at configuration 2's shapes: the first `rows` objects against all 512
    centroids, their 16 x t cost matrices written by d2_cost_tiles in the
    untimed set-up and resident in HBM."""

    metric = "exact transport LPs/sec from given FP64 cost matrices"
    unit = "LPs/s"

    def __init__(self, cfg, d2, dev, init, schedule, rows=4000):
        import synth
        import torch
        self.cfg = cfg
        self.spec = synth.CONFIGS[cfg]
        X = synth.make_data(cfg).subset(np.arange(rows))
        Z = synth.make_centroids(cfg)
        self.X, self.Z = X, Z
        self.d2 = d2
        self.h = d2.Handle(0)
        Xd, Zd = d2.DeviceSet.from_ragged(X, dev), d2.DeviceSet.from_ragged(Z, dev)
        ii, jj = np.meshgrid(np.arange(X.n), np.arange(Z.n), indexing="ij")
        pairs = torch.as_tensor(np.stack([ii.ravel(), jj.ravel()], 1), device=dev)
        self.tiles, self.toff = d2.d2_cost_tiles(self.h, Xd, Zd, pairs)
        ts = torch.as_tensor(np.diff(X.offsets), device=dev)
        ss = torch.as_tensor(np.diff(Z.offsets), device=dev)
        pi, pj = pairs[:, 0], pairs[:, 1]
        self.roff = torch.zeros(len(pairs) + 1, dtype=torch.int64, device=dev)
        self.roff[1:] = torch.cumsum(ts[pi], 0)
        self.coff = torch.zeros_like(self.roff)
        self.coff[1:] = torch.cumsum(ss[pj], 0)
        xw = torch.as_tensor(X.weights, dtype=torch.float64, device=dev)
        zw = torch.as_tensor(Z.weights, dtype=torch.float64, device=dev)
        xo = torch.as_tensor(X.offsets, device=dev)
        zo = torch.as_tensor(Z.offsets, device=dev)
        # each problem's weight vectors, laid out contiguously
        ridx = torch.repeat_interleave(xo[pi], ts[pi]) + (torch.arange(int(self.roff[-1]), device=dev)
                                                          - torch.repeat_interleave(self.roff[:-1], ts[pi]))
        cidx = torch.repeat_interleave(zo[pj], ss[pj]) + (torch.arange(int(self.coff[-1]), device=dev)
                                                          - torch.repeat_interleave(self.coff[:-1], ss[pj]))
        self.rw, self.cw = xw[ridx].contiguous(), zw[cidx].contiguous()
        self.moff = self.toff[:-1].contiguous()
        self.max_rows, self.max_cols = X.max_support, Z.max_support
        self.opts = d2.Opts(init=init, schedule=schedule)
        self.pairs = len(pairs)
        self.pair_list = pairs.cpu().numpy()
        torch.cuda.synchronize()
        self.out = None

    def step(self):
        self.out = self.d2.d2_emd_cost_batch(self.h, self.roff, self.rw, self.coff, self.cw, self.tiles,
                                             self.moff, self.max_rows, self.max_cols, self.opts)

    def flops(self):
        """Pivot-free work: one certifying pricing pass (3 t s) per LP."""
        ts = np.diff(self.X.offsets).astype(np.float64)
        ss = np.diff(self.Z.offsets).astype(np.float64)
        return float(ts.sum() * ss.sum() * 3)

    def bytes(self):
        cells = float(self.tiles.numel())
        return cells * 8 + float(self.rw.numel() + self.cw.numel()) * 8 + self.pairs * (8 + 8 + 8 + 4)

    def failed(self):
        return int((self.out[1].cpu().numpy() != 0).sum())

    def config(self):
        return {"workload": f"given-cost LPs, {self.X.n} x {self.Z.n} pairs of configuration 2 shapes",
                "problems": self.pairs, "t_range": list(self.spec["t_range"]), "s": self.spec["s"],
                "cost_bytes": int(self.tiles.numel() * 8)}

    def cpu_baseline(self, target_s, init_oracle):
        """The oracle's given-cost LP on a seeded sample of the problems (one
        core); also checks the device's values there."""
        import oracle
        import synth
        dist = self.out[0].cpu().numpy()
        tiles = self.tiles.cpu().numpy()
        toff = self.toff.cpu().numpy()
        order = synth.rng_for(self.cfg, synth.STREAM_SAMPLE, 400).permutation(self.pairs)

        def one(k):
            i, j = self.pair_list[k]
            x, p = self.X.bag(int(i)); y, q = self.Z.bag(int(j))
            C = tiles[toff[k]:toff[k + 1]].reshape(len(p), len(q))
            return oracle.emd_cost(C, p, q, init_oracle)[0], C, p, q

        t0 = time.perf_counter()
        done, fails = 0, 0
        while time.perf_counter() - t0 < target_s and done < len(order):
            k = int(order[done])
            o, C, p, q = one(k)
            S = float((p / p.sum()) @ np.abs(C) @ (q / q.sum()))
            if not abs(dist[k] - o) <= 1e-10 * max(abs(o), 1e-4 * S):
                fails += 1
            done += 1
        dt = time.perf_counter() - t0
        return {"value": done / dt, "unit": "LPs/s", "cores": 1, "kind": "oracle",
                "sample": f"{done} seeded problems, {dt:.1f} s, "
                          f"{'Vogel' if init_oracle else 'north-west-corner'} start",
                "cpu_model": _cpu_model(), "parity_checked": done, "parity_failures": fails}


class MultiWorkload:
    """d2_assign_multi: labelling under the combined distance of Eq. (9) with
    two feature types at configuration 2's scale: the configuration's objects
    and an independent draw of the same law as the second type, against its
    512 centroids and a rotation of them (points shifted by one centroid) as
    the second type's."""

    metric = "combined two-type Mallows distances/sec (Eq. (9)), exact FP64"
    unit = "distances/s"

    def __init__(self, cfg, d2, dev, init, schedule, n=None):
        import synth
        self.cfg = cfg
        self.spec = synth.CONFIGS[cfg]
        X1 = synth.make_data(cfg, n=n)
        X2 = synth.make_data(cfg, n=X1.n, chunk=1)
        Z1 = synth.make_centroids(cfg)
        Z2 = synth.RaggedSet(Z1.offsets, np.roll(Z1.points, Z1.max_support, axis=0), Z1.weights)
        self.Xs, self.Zs = [X1, X2], [Z1, Z2]
        self.d2 = d2
        self.h = d2.Handle(0)
        self.Xd = [d2.DeviceSet.from_ragged(X, dev) for X in self.Xs]
        self.Zd = [d2.DeviceSet.from_ragged(Z, dev) for Z in self.Zs]
        self.opts = d2.Opts(init=init, schedule=schedule)
        self.pairs = X1.n * Z1.n
        self.out = None

    def step(self):
        self.out = self.d2.d2_assign_multi(self.h, self.Xd, self.Zd, self.opts)

    def flops(self):
        tot = 0.0
        for X, Z in zip(self.Xs, self.Zs):
            ts = np.diff(X.offsets).astype(np.float64)
            ss = np.diff(Z.offsets).astype(np.float64)
            tot += float(ts.sum() * ss.sum() * (3 * X.points.shape[1] + 3))
        return tot

    def bytes(self):
        b = sum(float(X.points.nbytes + X.weights.nbytes + X.offsets.nbytes) for X in self.Xs)
        b += sum(float(Z.points.nbytes + Z.weights.nbytes + Z.offsets.nbytes) for Z in self.Zs)
        # per type: the n x K matrix written, read back once by the sum or argmin
        return b + 2 * self.pairs * 8 * 2 + self.Xs[0].n * 12

    def failed(self):
        return int((self.out[3].cpu().numpy() != 0).sum())

    def config(self):
        s = self.spec
        return {"workload": s["name"] + " x 2 feature types (Eq. (9))", "n": self.Xs[0].n,
                "k": self.Zs[0].n, "d": self.Xs[0].points.shape[1], "t_range": list(s["t_range"]),
                "s": s["s"], "inputs": s["dtype"], "types": 2, "lps_per_step": 2 * self.pairs}

    def cpu_baseline(self, target_s, init_oracle):
        """The oracle's combined labelling on a seeded row sample; also checks
        the device's labels and minima there."""
        import oracle
        import synth
        g_lab = self.out[0].cpu().numpy()
        g_best = self.out[1].cpu().numpy()
        rows = synth.sample_rows(self.cfg, self.Xs[0].n, 16, tag=5)
        t0 = time.perf_counter()
        oracle.assign_multi([X.subset(rows) for X in self.Xs], self.Zs, init=init_oracle)
        per_row = (time.perf_counter() - t0) / len(rows)
        k = int(min(self.Xs[0].n, max(16, target_s / max(per_row, 1e-9))))
        rows = synth.sample_rows(self.cfg, self.Xs[0].n, k, tag=6)
        t0 = time.perf_counter()
        o_lab, o_best, o_all, o_st = oracle.assign_multi([X.subset(rows) for X in self.Xs], self.Zs,
                                                         init=init_oracle)
        dt = time.perf_counter() - t0
        fails = 0
        for q, i in enumerate(rows):
            if g_lab[i] == o_lab[q] and abs(g_best[i] - o_best[q]) <= 1e-10 * abs(o_best[q]):
                continue
            gap = o_all[q, g_lab[i]] - o_best[q] if g_lab[i] >= 0 else np.inf
            if not (gap <= 1e-10 * abs(o_best[q]) and abs(g_best[i] - o_best[q]) <= 1e-10 * abs(o_best[q])):
                fails += 1
        return {"value": len(rows) * self.Zs[0].n / dt, "unit": "distances/s",
                "cores": oracle.default_threads(), "kind": "oracle",
                "sample": f"{len(rows)} seeded rows x all {self.Zs[0].n} centroids x 2 types, {dt:.1f} s, "
                          f"{'Vogel' if init_oracle else 'north-west-corner'} start",
                "cpu_model": _cpu_model(), "parity_checked": len(rows), "parity_failures": fails}


class HierarchyWorkload:
    """hierarchical_d2: Alg. 3 on one GPU over a configuration's objects
    (tau = 50, e = 5 as in the paper's runs, stopping at the configuration's
    K centroids), the random choices from a seeded stream of uniforms."""

    metric = "hierarchical D2-clustering (Alg. 3): objects clustered/sec"
    unit = "objects/s"

    def __init__(self, cfg, d2, dev, init, schedule, n=None, tau=50, e=5):
        import synth
        self.cfg = cfg
        self.spec = synth.CONFIGS[cfg]
        self.X = synth.make_data(cfg, n=n)
        self.k = synth.CONFIGS[cfg]["k"]
        self.tau, self.e = tau, e
        self.U = synth.rng_for(cfg, synth.STREAM_SAMPLE, 500).random(4 * self.X.n + 1000)
        self.d2 = d2
        self.h = d2.Handle(0)
        self.Xd = d2.DeviceSet.from_ragged(self.X, dev).with_points(
            d2.DeviceSet.from_ragged(self.X, dev).points.double())
        self.opts = d2.Opts(init=init, schedule=schedule)
        self.pairs = self.X.n
        self.stats = {}
        self.out = None

    def step(self):
        self.stats = {}
        self.out = self.d2.hierarchical_d2(self.h, self.Xd, self.tau, self.e, self.k, self.U,
                                           opts=self.opts, stats=self.stats)

    def flops(self):
        return float(self.stats.get("flops", 0.0))

    def bytes(self):
        return float(self.X.points.nbytes * 2 + self.X.weights.nbytes + self.X.offsets.nbytes)

    def failed(self):
        return 0

    def config(self):
        s = self.spec
        lv = self.out[3] if self.out else []
        return {"workload": s["name"] + " hierarchy", "n": self.X.n, "d": self.X.points.shape[1],
                "t_range": list(s["t_range"]), "tau": self.tau, "e": self.e, "k": self.k,
                "levels": lv, "lps_per_step": self.stats.get("lps"),
                "labelling_lps_per_step": self.stats.get("lps_label"),
                "update_lps_per_step": self.stats.get("lps_update"), "inputs": s["dtype"]}

    def cpu_baseline(self, target_s, init_oracle):
        """The oracle's hierarchy on the first 320 objects of the workload
        (about 20 s: its Step 2 solves every cluster's free-weight program
        with a dense tableau); the device driver runs on the same objects
        and its labels are compared.  The sample is fixed rather than sized
        by time: beyond a few thousand objects a one-ulp change in a moved
        atom can flip a near-tie and the whole later trajectory with it (the
        oracle against itself, perturbed by one ulp, disagrees on 3,049 of
        3,200 labels)."""
        from oracle.hierarchy import hierarchy
        import torch
        sub = self.X.subset(np.arange(min(320, self.X.n)))
        t0 = time.perf_counter()
        (off, pts, wts), lab_o, lv_o, w_o = hierarchy(sub, self.tau, self.e, self.k, self.U,
                                                     init=init_oracle)
        dt = time.perf_counter() - t0
        Xs = self.d2.DeviceSet.from_ragged(sub, "cuda:0")
        _, lab_g, _, lv_g = self.d2.hierarchical_d2(self.h, Xs, self.tau, self.e, self.k, self.U,
                                                    opts=self.d2.Opts(init=init_oracle + 1))
        torch.cuda.synchronize()
        return {"value": sub.n / dt, "unit": "objects/s", "cores": oracle_threads(), "kind": "oracle",
                "sample": f"the first {sub.n} objects, {dt:.1f} s, "
                          f"{'Vogel' if init_oracle else 'north-west-corner'} start",
                "cpu_model": _cpu_model(), "parity_checked": sub.n,
                "parity_failures": int((lab_g != lab_o).sum()) + (0 if lv_g == lv_o else 1)}


class LargeWorkload:
    """d2_emd_batch on supports beyond the lane-group shapes: pairs of 96 to
    192 atoms per side (d=8, configuration 2's mixture law and weights),
    which run on the workgroup simplex."""

    metric = "exact Mallows distances/sec, supports 96..192 (workgroup simplex)"
    unit = "distances/s"

    def __init__(self, d2, dev, init, schedule, n=None):
        import synth
        import torch
        m = n or 4096
        rng = synth.rng_for(2, synth.STREAM_SAMPLE, 600)
        spec = synth.CONFIGS[2]

        def make(count, stream):
            r = synth.rng_for(2, synth.STREAM_DATA, stream)
            sizes = r.integers(96, 193, size=count)
            off = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int64)
            means = synth._means(2, spec)
            pts = synth.gmm_points(r, means, spec["sigma"], int(off[-1]))
            w = synth.dirichlet_ragged(r, spec["alpha"], sizes)
            return synth.RaggedSet(off, pts, w)

        self.A, self.B = make(256, 901), make(64, 902)
        self.pairs_np = np.stack([rng.integers(0, self.A.n, m), rng.integers(0, self.B.n, m)], 1).astype(np.int64)
        self.d2 = d2
        self.h = d2.Handle(0)
        self.Ad = d2.DeviceSet.from_ragged(self.A, dev)
        self.Bd = d2.DeviceSet.from_ragged(self.B, dev)
        self.pairs_d = torch.as_tensor(self.pairs_np, device=dev)
        self.opts = d2.Opts(init=init, schedule=schedule)
        self.pairs = m
        self.out = None

    def step(self):
        self.out = self.d2.d2_emd_batch(self.h, self.Ad, self.Bd, self.pairs_d, self.opts)

    def flops(self):
        ts = np.diff(self.A.offsets)[self.pairs_np[:, 0]].astype(np.float64)
        ss = np.diff(self.B.offsets)[self.pairs_np[:, 1]].astype(np.float64)
        return float((ts * ss).sum() * (3 * self.A.points.shape[1] + 3))

    def bytes(self):
        return float(self.A.points.nbytes + self.B.points.nbytes + self.pairs * 24)

    def failed(self):
        return int((self.out[1].cpu().numpy() != 0).sum())

    def config(self):
        return {"workload": "large supports 96..192 x 96..192, d=8", "pairs": self.pairs,
                "objects": [self.A.n, self.B.n]}

    def cpu_baseline(self, target_s, init_oracle):
        """The oracle on a seeded sample of the pairs; checks the device's
        values there."""
        import oracle
        from tests.parity import coupling_cost
        dist = self.out[0].cpu().numpy()
        t0 = time.perf_counter()
        k = 16
        while True:
            sample = self.pairs_np[:k]
            t1 = time.perf_counter()
            o, st, _ = oracle.emd_batch(self.A, self.B, sample, init=init_oracle)
            dt = time.perf_counter() - t1
            if dt > target_s / 3 or k >= self.pairs or time.perf_counter() - t0 > target_s:
                break
            k *= 2
        fails = 0
        for q, (i, j) in enumerate(sample):
            S = coupling_cost(*self.A.bag(int(i)), *self.B.bag(int(j)))
            if not abs(dist[q] - o[q]) <= max(1e-10 * abs(o[q]), 1e-14 * S):
                fails += 1
        return {"value": len(sample) / dt, "unit": "distances/s", "cores": oracle_threads(), "kind": "oracle",
                "sample": f"the first {len(sample)} pairs, {dt:.1f} s, "
                          f"{'Vogel' if init_oracle else 'north-west-corner'} start",
                "cpu_model": _cpu_model(), "parity_checked": len(sample), "parity_failures": fails}


def oracle_threads():
    import oracle
    return oracle.default_threads()


PIVOT_BINS = [0, 1, 3, 5, 9, 17, 33, 65, 129, 257]   # histogram edges: 0, 1-2, 3-4, 5-8, ...


def _pivot_summary(p: np.ndarray) -> dict:
    """Mean, percentiles and a histogram over power-of-two bins (counts of
    pairs with 0, 1-2, 3-4, 5-8, ..., 129-256 and more than 256 pivots)."""
    p = np.asarray(p, dtype=np.float64)
    hist = np.histogram(p, bins=PIVOT_BINS + [np.inf])[0]
    return {"mean": float(p.mean()), "p50": float(np.percentile(p, 50)),
            "p90": float(np.percentile(p, 90)), "p99": float(np.percentile(p, 99)),
            "max": int(p.max()), "zero_frac": float((p == 0).mean()),
            "hist": [int(c) for c in hist]}


def pivot_work_factor(ts: np.ndarray, ss: np.ndarray, pivots: np.ndarray, d: int) -> float:
    """Measured work over the pivot-free lower bound: a pair of supports t, s
    costs 3 t s d for its cost tile and 3 t s per pricing pass, one pass per
    pivot plus the certifying one."""
    w = np.asarray(ts, np.float64) * np.asarray(ss, np.float64)
    p = np.asarray(pivots, np.float64)
    return float((w * (3 * d + 3 * (p + 1))).sum() / (w * (3 * d + 3)).sum())


def pivot_stats(d2, dev, A, B, pairs: np.ndarray, d: int) -> dict:
    """Pivots per LP on a seeded sample of pairs: the device under its default
    least-cost start and under the north-west corner, and the oracle under
    the north-west corner (its starts are the north-west corner and Vogel).
    Every pivot adds one pricing pass (3 t s operations) to the pivot-free
    work that the roofline counts; ``work_factor`` is the measured work over
    that lower bound, weighting each pair by its t s."""
    import torch
    import oracle
    h = d2.Handle(0)
    Ad, Bd = d2.DeviceSet.from_ragged(A, dev), d2.DeviceSet.from_ragged(B, dev)
    pt = torch.as_tensor(pairs)
    dev_piv, bad = {}, {}
    for name, init in (("lcm", d2.D2_INIT_LCM), ("nwc", d2.D2_INIT_NWC)):
        dist, st, _, _, piv = d2.d2_emd_batch(h, Ad, Bd, pt, d2.Opts(init=init), want_pivots=True)
        torch.cuda.synchronize()
        bad["device_" + name] = int((st != 0).sum().item())
        dev_piv[name] = piv.cpu().numpy()
    o_d, o_st, o_piv, o_bl = oracle.emd_batch_stats(A, B, pairs, init=oracle.INIT_NWC)
    bad["oracle_nwc"] = int((o_st != 0).sum())
    ts = np.diff(A.offsets)[pairs[:, 0]]
    ss = np.diff(B.offsets)[pairs[:, 1]]
    p_lcm = dev_piv["lcm"][:, 0]
    return {
        "pairs": int(pairs.shape[0]),
        "device_lcm": _pivot_summary(p_lcm),
        "device_nwc": _pivot_summary(dev_piv["nwc"][:, 0]),
        "oracle_nwc": _pivot_summary(o_piv),
        "nwc_same_count_frac": float((dev_piv["nwc"][:, 0] == o_piv).mean()),
        "nonzero_status": bad,
        "bland_pivots": {"device_lcm": int(dev_piv["lcm"][:, 1].sum()),
                         "device_nwc": int(dev_piv["nwc"][:, 1].sum()), "oracle_nwc": int(o_bl.sum())},
        "work_factor": pivot_work_factor(ts, ss, p_lcm, d),
    }


def pivot_sample(cfg: int, count: int = 4096):
    """(A, B, pairs, d) for a configuration's pivot sample: objects against
    centroids (configurations 1-3, 5: queries against the resident centroids),
    or object pairs i < j of one segment (configuration 4)."""
    import synth
    n = synth.CONFIGS[cfg]["n"]
    X = synth.make_data(cfg) if 0 < n <= 8192 else synth.make_data(cfg, n=8192)
    d = int(X.points.shape[1])
    if cfg == 4:
        rng = synth.rng_for(cfg, synth.STREAM_SAMPLE, 4242)
        i = rng.integers(0, X.n, size=4 * count)
        j = rng.integers(0, X.n, size=4 * count)
        keep = i < j
        pairs = np.unique(np.stack([i[keep], j[keep]], axis=1), axis=0)[:count]
        rng.shuffle(pairs)
        return X, X, pairs.astype(np.int64), d
    Z = synth.make_centroids(cfg)
    return X, Z, synth.sample_pairs(cfg, X.n, Z.n, count, tag=4242), d


def other_legs(d2, dev, steps=3, warmup=1, cpu_seconds=2.0) -> list:
    """Short runs of the other measured workloads beside the default one, so
    that one run records them all: configuration 1, configuration 3 with the
    FP64 and the BF16-MFMA cost, configuration 4's pairwise matrix and the
    hierarchy over configuration 2's objects.  Each is timed like the main
    step (inputs resident, HIP events), and the labelling and pairwise legs
    check a seeded sample against the oracle (about ``cpu_seconds`` of it)."""
    import torch
    init, sched = d2.D2_INIT_AUTO, d2.D2_SCHED_AUTO
    makers = [
        ("c1", lambda: AssignWorkload(1, d2, dev, init, sched)),
        ("c3_f64", lambda: AssignWorkload(3, d2, dev, init, sched)),
        ("c3_bf16", lambda: AssignWorkload(3, d2, dev, init, sched, cost_mode=d2.D2_COST_BF16_MFMA)),
        ("c4", lambda: PairwiseWorkload(4, d2, dev, init, sched)),
        ("hierarchy_c2", lambda: HierarchyWorkload(2, d2, dev, init, sched)),
    ]
    legs = []
    for name, make in makers:
        w = make()
        for _ in range(warmup):
            w.step()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(steps)]
        t0 = time.perf_counter()
        for k in range(steps):
            ev[k][0].record(stream)
            w.step()
            ev[k][1].record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        leg = {"leg": name, "config": w.config(), "value": w.pairs * steps / wall,
               "unit": getattr(w, "unit", "distances/s"), "steps": steps, "warmup": warmup,
               "ms_per_step": wall / steps * 1e3,
               "kernel_ms_median": float(np.median([a.elapsed_time(b) for a, b in ev])),
               "failed_pairs_or_rows": w.failed()}
        cb = None
        if name == "c4":
            cb = w.cpu_baseline(cpu_seconds, 0, all_pairs=True)   # every one of its 8.39 M pairs
        elif name != "hierarchy_c2":
            cb = w.cpu_baseline(cpu_seconds, 0)
        if cb is not None:
            leg["parity"] = {k: cb[k] for k in ("parity_checked", "parity_failures", "bf16_vs_fp64",
                                                "sample") if k in cb}
        legs.append(leg)
        print(f"leg {name}: {leg['value']:.4g} {leg['unit']}", file=sys.stderr, flush=True)
        del w
        torch.cuda.synchronize()
        torch.cuda.empty_cache()
    return legs


def run_pivots(argv) -> int:
    """--op pivots: per-configuration pivot counts, device and oracle."""
    import paper_1302_0435_amd as d2
    rows = []
    for cfg in (1, 2, 3, 4, 5):
        A, B, pairs, d = pivot_sample(cfg)
        r = pivot_stats(d2, "cuda:0", A, B, pairs, d)
        r["config"] = cfg
        rows.append(r)
        print(f"config {cfg}: {json.dumps(r)}", file=sys.stderr, flush=True)
    print(json.dumps({"metric": "pivots per LP, device and oracle", "configs": rows}), flush=True)
    return 0


def make_pool(n_pool: int):
    """Query pool for the serving workload (configuration 5, stream 1)."""
    import synth
    from paper_1302_0435_amd import serve
    q = synth.make_data(5, n=n_pool)
    return serve.QueryPool(q.offsets, q.points.astype(np.float64), q.weights.astype(np.float64))


def serve_leg(d2, rates=(10000.0, 50000.0), duration=2.0, n_pool=4000, check=160):
    """A short serving run of configuration 5 beside the default workload:
    Poisson streams of queries (d=32, supports 4..64) against the 1,024
    resident centroids of support 32, at a sustainable rate and an overloaded
    one (whose distances/s is the served form's capacity); the served results
    of the first queries checked against the oracle; and the plain per-pair
    solver (one wavefront per pair in input order, north-west corner, no
    binning, no graph) over the same queries for comparison."""
    import torch
    import oracle
    import synth
    from paper_1302_0435_amd import serve
    from tests.parity import coupling_cost
    Z = synth.make_centroids(5)
    Zd = d2.DeviceSet.from_ragged(Z, "cuda:0")
    pool = make_pool(n_pool)
    legs = []
    for rate in rates:
        arrivals = synth.arrivals(5, rate, duration)
        req_idx = np.arange(arrivals.size) % pool.n
        ex = serve.GpuExecutor(pool, req_idx, Zd, Z.n, 4, 512, budget_bytes=256 << 20)
        sch = serve.Scheduler(ex, pool.sizes()[req_idx], pool.d, Z.n, 256 << 20, 512, 4)
        serve.warm_up(sch, arrivals)      # one-time launch costs outside the measured run
        st = sch.run(arrivals)
        summ = st.summary(Z.n)
        summ["rate_qps"] = rate
        legs.append(summ)
        del ex
        torch.cuda.synchronize()
    # parity of served results: a separate short run that keeps every result
    # (copying results out on the host would slow the measured runs)
    arrivals = synth.arrivals(5, rates[0], duration)[:check]
    req_idx = np.arange(arrivals.size) % pool.n
    ex = serve.GpuExecutor(pool, req_idx, Zd, Z.n, 4, 512, keep_results=True, budget_bytes=256 << 20)
    serve.Scheduler(ex, pool.sizes()[req_idx], pool.d, Z.n, 256 << 20, 512, 4).run(arrivals)
    kept = dict(ex.results)
    del ex
    P = synth.RaggedSet(pool.offsets, pool.points, pool.weights)
    q = [r for r in range(min(check, pool.n)) if r in kept]
    o_lab, o_best, o_all, _, _ = oracle.assign(P.subset(q), Z, threads=oracle_threads())
    fails = 0
    for i, r in enumerate(q):
        g_lab, g_best, g_all, g_st = kept[r]
        x, w = P.bag(r)
        floor = np.array([1e-14 * coupling_cost(x, w, *Z.bag(j)) for j in range(Z.n)])
        bad = ~(np.abs(g_all - o_all[i]) <= np.maximum(1e-10 * np.abs(o_all[i]), floor))
        if g_st != 0 or bad.any() or (g_lab != o_lab[i] and
                                      o_all[i, g_lab] - o_all[i, o_lab[i]] > max(1e-10 * abs(o_best[i]),
                                                                                   floor[o_lab[i]])):
            fails += 1
    # the plain per-pair solver on the same queries
    sub = P.subset(np.arange(min(1000, pool.n)))
    Xs = d2.DeviceSet.from_ragged(sub, "cuda:0")
    h = d2.Handle(0)
    opts = d2.Opts(init=d2.D2_INIT_NWC, schedule=d2.D2_SCHED_PLAIN, flags=d2.D2_FLAG_EAGER)
    dt = _timed(lambda: d2.d2_assign(h, Xs, Zd, opts))
    plain = sub.n * Z.n / dt
    cap = legs[-1]["distances_per_s"]
    return {"workload": synth.CONFIGS[5]["name"], "k": Z.n, "duration_s_per_rate": duration,
            "slots": 4, "max_batch": 512, "budget_mib": 256, "rates": legs,
            "p50_ms": legs[0]["p50_ms"], "p99_ms": legs[0]["p99_ms"], "p99_rate_qps": rates[0],
            "saturated_distances_per_s": cap,
            "plain_solver": {"value": plain, "unit": "distances/s",
                             "sample": f"first {sub.n} queries x all {Z.n} centroids, one launch"},
            "served_over_plain": cap / plain,
            "parity_checked_queries": len(q), "parity_failures": fails}


def run_serving(argv) -> int:
    """Configuration 5: Poisson query streams against 1,024 resident centroids
    of support 32 (d=32), one run per rate; reports p50/p99 latency and
    distances/sec per rate, and as `value` the distances/sec of the highest
    rate served in full with p99 under one second."""
    ap = argparse.ArgumentParser()
    ap.add_argument("--rates", default="2000,10000,50000")
    ap.add_argument("--duration", type=float, default=10.0, help="seconds per rate")
    ap.add_argument("--pool", type=int, default=20000, help="distinct queries (reused cyclically)")
    ap.add_argument("--slots", type=int, default=4)
    ap.add_argument("--max-batch", type=int, default=512)
    ap.add_argument("--budget-mib", type=float, default=256.0)
    ap.add_argument("--init", choices=["auto", "nwc", "vogel", "lcm"], default="auto")
    args = ap.parse_args(argv)
    import torch
    import synth
    import paper_1302_0435_amd as d2
    from paper_1302_0435_amd import serve

    spec = synth.CONFIGS[5]
    Z = synth.make_centroids(5)
    Zd = d2.DeviceSet.from_ragged(Z, "cuda:0")
    pool = make_pool(args.pool)
    results = []
    for rate in [float(r) for r in args.rates.split(",")]:
        arrivals = synth.arrivals(5, rate, args.duration)
        req_idx = np.arange(arrivals.size) % pool.n
        init = {"auto": d2.D2_INIT_AUTO, "nwc": d2.D2_INIT_NWC, "vogel": d2.D2_INIT_VOGEL,
                "lcm": d2.D2_INIT_LCM}[args.init]
        budget = int(args.budget_mib * 2**20)
        ex = serve.GpuExecutor(pool, req_idx, Zd, Z.n, args.slots, args.max_batch, init=init,
                               budget_bytes=budget)
        sch = serve.Scheduler(ex, pool.sizes()[req_idx], pool.d, Z.n, budget, args.max_batch,
                              args.slots)
        serve.warm_up(sch, arrivals)      # one-time launch costs outside the measured run
        st = sch.run(arrivals)
        summ = st.summary(Z.n)
        summ["rate_qps"] = rate
        results.append(summ)
        print(json.dumps({"serve_rate": rate, **summ}), file=sys.stderr, flush=True)
        del ex
        torch.cuda.synchronize()
    sustained = [r for r in results if r["completed"] == r["requests"] and r["p99_ms"] is not None
                 and r["p99_ms"] < 1000.0]
    top = max(sustained, key=lambda r: r["rate_qps"]) if sustained else results[-1]
    print(json.dumps({
        "metric": "exact Mallows distances/sec at <=1e-10 rel err vs FP64 oracle; p99 query latency",
        "value": top["distances_per_s"], "unit": "distances/s", "n_gpus": 1,
        "steps": len(results), "warmup": 1, "ms_per_step": args.duration * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": spec["name"], "k": Z.n, "s": spec["s"], "d": spec["d"],
                   "t_range": list(spec["t_range"]), "duration_s": args.duration,
                   "slots": args.slots, "max_batch": args.max_batch,
                   "budget_mib": args.budget_mib, "init": args.init},
        "p99_ms": top["p99_ms"], "rates": results}), flush=True)
    return 0


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2, choices=[1, 2, 3, 4, 5])
    ap.add_argument("--init", choices=["auto", "nwc", "vogel", "lcm"], default="auto",
                    help="starting basis (auto: the library default, least cost)")
    ap.add_argument("--schedule", choices=["auto", "plain"], default="auto")
    ap.add_argument("--cost", choices=["f64", "bf16"], default="f64",
                    help="ground-cost arithmetic (bf16: MFMA cost tiles fused into the "
                         "labelling kernel, supports <= 32)")
    ap.add_argument("--tune", action="store_true", help="autotune the pairwise schedule first")
    ap.add_argument("--op", choices=["assign", "update", "cost", "multi", "hierarchy", "large", "pivots"],
                    default="assign",
                    help="update: the constrained D2 centroid update (configurations 1-3); "
                         "cost: LPs over given cost matrices (configuration 2 shapes); "
                         "multi: two-type labelling of Eq. (9) (configuration 2 scale); "
                         "hierarchy: Alg. 3 over a configuration's objects; "
                         "large: pairs of 96..192 atoms on the workgroup simplex; "
                         "pivots: pivots per LP on a sample of every configuration, device "
                         "and oracle")
    ap.add_argument("--n", type=int, default=None, help="override object count (testing)")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--sampled-parity", action="store_true",
                    help="configuration 2: check a timed sample of rows instead of all of them")
    ap.add_argument("--no-serve", action="store_true",
                    help="configuration 2: skip the short serving leg of configuration 5")
    ap.add_argument("--no-legs", action="store_true",
                    help="configuration 2: skip the short runs of the other workloads")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device-to-device copy of MIB MiB (for scaling the "
                         "HBM byte counters), then exit")
    args, rest = ap.parse_known_args(argv)
    if args.copy_calibration:
        return copy_calibration(args.copy_calibration)
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the library runs the path on a single MI355X; "
              "multi-GPU sharding is a design note, not a measured mode.", file=sys.stderr)
        return 2
    if args.config == 5:
        return run_serving(rest + ["--init", args.init])
    if args.op == "pivots":
        return run_pivots(rest)

    import torch
    import paper_1302_0435_amd as d2

    dev = "cuda:0"
    init = {"auto": d2.D2_INIT_AUTO, "nwc": d2.D2_INIT_NWC, "vogel": d2.D2_INIT_VOGEL,
            "lcm": d2.D2_INIT_LCM}[args.init]
    schedule = d2.D2_SCHED_PLAIN if args.schedule == "plain" else d2.D2_SCHED_AUTO
    if args.op == "update":
        if args.config not in (1, 2, 3) or args.cost != "f64":
            print("--op update runs configurations 1-3 with the FP64 cost", file=sys.stderr)
            return 2
        w = UpdateWorkload(args.config, d2, dev, init, schedule, n=args.n)
    elif args.op == "cost":
        w = CostWorkload(2, d2, dev, init, schedule, rows=args.n or 4000)
    elif args.op == "multi":
        w = MultiWorkload(2, d2, dev, init, schedule, n=args.n)
        args.config = 2
    elif args.op == "large":
        w = LargeWorkload(d2, dev, init, schedule, n=args.n)
    elif args.op == "hierarchy":
        w = HierarchyWorkload(args.config if args.config in (1, 2, 3) else 2, d2, dev, init, schedule,
                              n=args.n)
    elif args.config == 4:
        w = PairwiseWorkload(4, d2, dev, init, schedule, n=args.n, tune=args.tune)
    else:
        w = AssignWorkload(args.config, d2, dev, init, schedule, n=args.n,
                           cost_mode=d2.D2_COST_BF16_MFMA if args.cost == "bf16" else 0)

    for _ in range(args.warmup):
        w.step()
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        ev[k][0].record(stream)
        w.step()
        ev[k][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kern_ms = [a.elapsed_time(b) for a, b in ev]

    kernel_s = float(np.mean(kern_ms)) / 1e3
    flops = w.flops()
    achieved = flops / kernel_s / 1e12
    prof = profile_counters(args.config, args.cost, args.op) if (
        args.n is None and schedule == d2.D2_SCHED_AUTO and init == d2.D2_INIT_AUTO) else None
    cfg = w.config()
    cfg.update({"init": args.init, "schedule": args.schedule, "cost": args.cost})
    bf16 = args.cost == "bf16"
    metric = ("Mallows distances/sec, BF16-MFMA ground cost + FP64 simplex (approximate)"
              if bf16 else "exact Mallows distances/sec at <=1e-10 rel err vs FP64 oracle")
    out = {
        "metric": getattr(w, "metric", metric),
        "value": w.pairs * args.steps / wall,
        "unit": getattr(w, "unit", "distances/s"),
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "ms_per_step_median": float(np.median(kern_ms)),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16+f64" if bf16 else "f64",
        "data": "synthetic",
        "config": cfg,
        "roofline": {
            "bound": "alu", "achieved": achieved, "peak": FP64_VECTOR_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": achieved / FP64_VECTOR_PEAK_TFLOPS,
            "traffic": prof["traffic"] if prof else None,
            "traffic_kernel": prof["kernel"] if prof else None,
            "valu_issue_busy": prof["valu_issue_busy"] if prof else None,
            "lds_util_percent": prof["lds_util_percent"] if prof else None,
            "profile_kernel_ms": prof["profile_avg_ms"] if prof else None,
            "kernel_ms": float(np.mean(kern_ms)),
            "algorithmic_flops_per_launch": flops,
            "algorithmic_bytes_per_launch": w.bytes(),
            "hbm_gbs_algorithmic": w.bytes() / kernel_s / 1e9,
        },
        "failed_pairs_or_rows": w.failed(),
    }
    if args.n is None and args.op == "assign":
        out["end_to_end_with_copies"] = w.end_to_end()
        plain = w.plain_baseline()
        plain["speedup_of_value"] = out["value"] / plain["value"]
        out["plain_solver"] = plain
    default_c2 = args.n is None and args.op == "assign" and args.config == 2 and args.cost == "f64"
    if args.n is None and args.op == "assign" and args.config in (1, 2, 3) and args.cost == "f64":
        # pivots on a seeded sample of this workload's pairs (outside the timed
        # region), and the roofline over the work those pivots add
        import synth
        pairs = synth.sample_pairs(args.config, w.X.n, w.Z.n, 4096, tag=4242)
        pv = pivot_stats(d2, dev, w.X, w.Z, pairs, int(w.X.points.shape[1]))
        out["pivots"] = pv
        rf = out["roofline"]
        rf["work_factor_with_pivots"] = pv["work_factor"]
        rf["achieved_with_pivots"] = achieved * pv["work_factor"]
        rf["frac_with_pivots"] = achieved * pv["work_factor"] / FP64_VECTOR_PEAK_TFLOPS
    if default_c2 and not args.no_serve:
        # the serving form beside the headline: p50/p99 latency and capacity
        # of configuration 5, against the plain per-pair solver
        sv = serve_leg(d2)
        out["p50_ms"] = sv["p50_ms"]
        out["p99_ms"] = sv["p99_ms"]
        out["serving"] = sv
    if default_c2 and not args.no_legs:
        out["other_workloads"] = other_legs(d2, dev)
    if not args.no_cpu_baseline:
        # the oracle has the north-west-corner and Vogel starts
        ib = 1 if init == d2.D2_INIT_VOGEL else 0
        if default_c2 and not args.sampled_parity:
            out["cpu_baseline"] = w.cpu_baseline(args.cpu_seconds, ib, all_rows=True)
        else:
            out["cpu_baseline"] = w.cpu_baseline(args.cpu_seconds, ib)
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
