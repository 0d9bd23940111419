"""Throughput of the masked-L2 patch search on one MI355X.

One step runs the whole hot path over one synthetic workload: fill front and
target extraction, the SFC multi-index build (byte codes, covariance, Jacobi,
int8 basis, MFMA projection, keys, radix sort), the index query of every
front target, and the full float32 scan plus the reduced-precision (bf16
MFMA) scan of every front target. `value` is front queries answered per
second by that whole step; the per-form rates are reported beside it.

The default workload is the 1024x1024 RGB image (n ~ 0.9e6). After its timed
steps, one pass over the 512^3 volume (n ~ 1.25e8) reports the index query
rate over its whole front and the float32 scan rate on a seeded sample of
4096 front targets (`n1e8`), and 16 uneven images (sides 256-1024, 1-3
channels) report the batched, graph-replayed float32 scan (`batch`);
`--workload config5` times that batch over 64 images (sides 256-2048).

  python bench.py [--steps K] [--warmup W] [--workload config2] [--no-cpu-baseline]
                  [--no-n1e8] [--no-batch] [--calib-copy]

Prints one JSON line. Only N=1 is supported: this build runs on one GPU.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Published MI355X peaks. FP32 vector: 256 CU x 128 lanes x 2 flop x 2.4 GHz.
PEAK_FP32_VALU = 157.3   # TFLOP/s
PEAK_BF16_MFMA = 2500.0  # TFLOP/s, dense
PEAK_HBM = 8000.0        # GB/s

WORKLOADS = {
    "config1": dict(gen="config1", K=9, D=8, L=4, key_bits=8, window=32, curve="morton",
                    scan_sample=0, bf16=True, label="config1_256sq_gray_hole32_K9 (n~6e4)"),
    "config2": dict(gen="config2", K=9, D=8, L=4, key_bits=21, window=32, curve="morton",
                    scan_sample=0, bf16=True, label="config2_1024sq_rgb_blobs10_K9 (n~0.9e6)"),
    "config3": dict(gen="config3", K=7, D=10, L=6, key_bits=8, window=32, curve="hilbert",
                    scan_sample=4096, bf16=True, label="config3_256cube_tomo_voids5_K7 (n~1.4e7)"),
    "config4": dict(gen="config4", K=5, D=8, L=4, key_bits=8, window=32, curve="morton",
                    scan_sample=4096, bf16=False,
                    label="config4_512cube_phantom_u16_K5 (n~1.25e8)"),
    "config5": dict(gen="config5", K=9, n_images=64, sides=(256, 2048),
                    label="config5_64_images_256-2048_C1-3_K9"),
}


def cpu_model():
    try:
        for ln in open("/proc/cpuinfo"):
            if ln.startswith("model name"):
                return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def source_hash(names):
    h = hashlib.sha256()
    for n in names:
        with open(os.path.join(ROOT, "paper_1712_06326_amd", "csrc", n), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def load_traffic(kernel_key, workload, src_hash):
    """HBM bytes per launch from the committed counter summary, if it was
    taken on the current source of the kernel."""
    p = os.path.join(ROOT, "profiles", f"{kernel_key}_{workload}_traffic.json")
    if not os.path.exists(p):
        return None
    d = json.load(open(p))
    if d.get("source_hash") != src_hash:
        return None
    return d.get("bytes_per_launch")


class Workload:
    """Synthetic volume on the device plus its front targets."""

    def __init__(self, name, torch, native, synth):
        self.name, self.cfg = name, WORKLOADS[name]
        t0 = time.time()
        data = getattr(synth, self.cfg["gen"])()
        log(f"generated {self.cfg['label']} in {time.time() - t0:.1f}s")
        self.vol_h, self.mask_h = data["volume"], data["mask"]
        dev = torch.device("cuda:0")
        self.vol = torch.from_numpy(self.vol_h).to(dev)
        self.mask = torch.from_numpy(self.mask_h).to(dev)
        self.K = self.cfg["K"]
        self.opts = dict(key_bits=self.cfg["key_bits"], window=self.cfg["window"],
                         curve=self.cfg["curve"])
        f = native.fill_front(self.mask)
        self.Q = int(f.numel())
        k = self.cfg["scan_sample"]
        if k and k < self.Q:
            sel = np.sort(np.random.default_rng(5).choice(self.Q, k, replace=False))
            self.sel = torch.from_numpy(sel).to(dev)
        else:
            self.sel = None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=5)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--workload", default="config2", choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-n1e8", action="store_true", help="skip the n~1.25e8 pass")
    ap.add_argument("--no-batch", action="store_true", help="skip the batched-images pass")
    ap.add_argument("--no-inpaint", action="store_true", help="skip the whole-inpainting runs")
    ap.add_argument("--cpu-sample", type=int, default=48, help="oracle full-scan queries timed")
    ap.add_argument("--calib-copy", action="store_true",
                    help="also run one 512 MiB device copy (HBM counter calibration)")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)

    import torch
    from paper_1712_06326_amd import native, synth

    stream = torch.cuda.current_stream()

    def ev():
        e = torch.cuda.Event(enable_timing=True)
        e.record(stream)
        return e

    if args.workload == "config5":
        cfg = WORKLOADS["config5"]
        res = batch_pass(torch, native, synth, ev, cfg["n_images"], cfg["sides"], args.steps,
                         args.warmup)
        line = {
            "metric": "queries/s at n=1e6,1e8 (SFC index vs GPU brute force), argmin agreement %",
            "value": res["qps"], "unit": "queries/s", "n_gpus": 1, "steps": args.steps,
            "warmup": args.warmup, "ms_per_step": res["ms_per_replay"],
            "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
            "data": "synthetic",
            "config": {"workload": cfg["label"], "images": cfg["n_images"], "K": cfg["K"],
                       "queries": res["queries"]},
            "forms": res}
        print(json.dumps(line), flush=True)
        return

    w = Workload(args.workload, torch, native, synth)
    cfg, K = w.cfg, w.K

    def step(record, ktimes):
        e = [ev()]
        f = native.fill_front(w.mask)
        t, m = native.extract_targets(w.vol, w.mask, K, f)
        e.append(ev())
        ix = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], timing=True,
                          **w.opts)
        e.append(ev())
        # the index query runs without the library's timing events (its
        # kernels are timed separately after the steps); the scans with them
        ix.set_timing(False)
        bi_x, bc_x = ix.query(t, m, "index")
        ix.set_timing(True)
        e.append(ev())
        ts, ms = (t, m) if w.sel is None else (t[w.sel].contiguous(), m[w.sel].contiguous())
        bi_s, bc_s = ix.query(ts, ms, "fp32")
        e.append(ev())
        out = dict(n=ix.info.n, t=ts, m=ms, bi_x=bi_x, bc_x=bc_x, bi_s=bi_s, bc_s=bc_s)
        if cfg["bf16"]:
            bi_r, bc_r = ix.query(ts, ms, "bf16")
            e.append(ev())
        # the library keeps every timed launch of the step until this read
        # (after the last mark, so no phase waits on the host); the bf16
        # scan's float32 fallback is timed as "scan_fp32_kernel<fallback>"
        kt = dict(ix.kernel_times())
        if cfg["bf16"]:
            out.update(bi_r=bi_r, bc_r=bc_r, fallback=ix.fallbacks(), tiles=ix.filter_tiles())
        if record is not None:
            record.append(e)
            ktimes.append(kt)
        ix.close()
        return out

    # the index's recall and acceleration error against the window width
    # (Section III.D's candidate-set trade-off), from the window autotuner
    # on a seeded sample of 1024 front targets; the timed steps keep the
    # workload's window
    window_trials = None
    if cfg.get("D"):
        fz = native.fill_front(w.mask)
        tz, mz = native.extract_targets(w.vol, w.mask, K, fz)
        kz = min(1024, w.Q)
        sz = torch.from_numpy(np.sort(np.random.default_rng(3).choice(w.Q, kz, replace=False))).cuda()
        iz = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], **w.opts)
        wz, window_trials = iz.autotune_window(tz[sz].contiguous(), mz[sz].contiguous(), 0.9, -1.0)
        iz.close()
        del fz, tz, mz
        log(f"window autotuner: W={wz} reaches recall 0.9 on the sample")

    # autotune the float32 scan's tile shape once on this workload (the
    # choice is remembered for every later handle of the same shape)
    f0 = native.fill_front(w.mask)
    t0_, m0_ = native.extract_targets(w.vol, w.mask, K, f0)
    if w.sel is not None:
        t0_, m0_ = t0_[w.sel].contiguous(), m0_[w.sel].contiguous()
    ix0 = native.Index(w.vol, w.mask, K)
    chosen = ix0.autotune(t0_, m0_)
    ix0.close()
    del f0, t0_, m0_
    log(f"autotuned float32-scan shape: {chosen}")
    for _ in range(args.warmup):
        step(None, None)
    torch.cuda.synchronize()
    marks, ktimes = [], []
    t_start = time.perf_counter()
    for _ in range(args.steps):
        res = step(marks, ktimes)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_start
    ms_step = 1e3 * wall / args.steps
    ph = np.array([[a.elapsed_time(b) for a, b in zip(mk[:-1], mk[1:])] for mk in marks]).mean(0)
    kavg = {k: float(np.mean([kt[k][1] / kt[k][0] for kt in ktimes])) for k in ktimes[0]}
    # the index query's kernels: three timed runs of the same query on a
    # handle of the same build, after the steps
    if cfg.get("D"):
        fx = native.fill_front(w.mask)
        tx, mx = native.extract_targets(w.vol, w.mask, K, fx)
        ixt = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], timing=True,
                           **w.opts)
        ixt.query(tx, mx, "index")
        ixt.kernel_times()
        for _ in range(3):
            ixt.query(tx, mx, "index")
        kavg.update({k: v[1] / v[0] for k, v in ixt.kernel_times().items()})
        # the same batch ten times in a row without timing events: the host
        # stays ahead, so this is the query's own rate (the step's phase
        # also holds the host's launch latency after the build)
        ixt.set_timing(False)
        a = ev()
        for _ in range(10):
            ixt.query(tx, mx, "index")
        b = ev()
        torch.cuda.synchronize()
        index_b2b_ms = a.elapsed_time(b) / 10
        ixt.close()
        del fx, tx, mx
    else:
        index_b2b_ms = None
    Q, n = w.Q, res["n"]
    Qs = int(res["m"].shape[0])
    m_h = res["m"].cpu().numpy()
    C = w.vol_h.shape[-1]
    P = K ** (w.mask_h.ndim) * C
    known_elems = float(m_h.sum()) * C

    # index vs float32 scan on the scanned queries: recall@1, acceleration error
    bi_x, bc_x = res["bi_x"], res["bc_x"]
    if w.sel is not None:
        bi_x, bc_x = bi_x[w.sel], bc_x[w.sel]
    bi_x, bc_x = bi_x.cpu().numpy(), bc_x.cpu().numpy()
    bi_s, bc_s = res["bi_s"].cpu().numpy(), res["bc_s"].cpu().numpy()
    recall = float(np.mean(bi_x == bi_s))
    # equal cost counts too: flat or repeated texture has several optimal patches
    cost_recall = float(np.mean(bc_x.view(np.uint32) == bc_s.view(np.uint32)))
    ok = bc_s > 0
    ae = float(np.mean(np.sqrt(bc_x[ok].astype(np.float64)) / np.sqrt(bc_s[ok]) - 1.0)) * 100

    # rooflines of the dominant kernels, from their own launch durations
    scan_flops = 3.0 * known_elems * n
    roofs = {"scan_fp32_kernel": {
        "bound": "alu", "kernel": "scan_fp32_kernel",
        "achieved": scan_flops / (kavg["scan_fp32_kernel"] * 1e-3) / 1e12,
        "peak": PEAK_FP32_VALU, "unit": "TFLOP/s",
        "traffic": load_traffic("scan_fp32", args.workload, source_hash(["k_scan.hip"])),
        "work_per_launch": f"{scan_flops:.4g} flop = 3 x {known_elems:.0f} known elements x n"}}
    if cfg["bf16"]:
        # the filter GEMM's useful width: C codes plus 2 norm columns per pixel
        kd = K ** w.mask_h.ndim
        gemm_flops = 2.0 * kd * (C + 2) * n * Qs
        for k in ("filter_kernel<list>", "filter_kernel<min>"):
            if k in kavg:
                key = "filter_bf16_" + k[len("filter_kernel<"):-1]
                roofs[k] = {
                    "bound": "mfma", "kernel": k,
                    "achieved": gemm_flops / (kavg[k] * 1e-3) / 1e12,
                    "peak": PEAK_BF16_MFMA, "unit": "TFLOP/s",
                    "traffic": load_traffic(key, args.workload, source_hash(["k_mfma_scan.hip"])),
                    "work_per_launch": f"{gemm_flops:.4g} flop = 2 x K^d(C+2) x n x Q"}
    dom = max(roofs, key=lambda k: kavg.get(k, 0.0))
    for r in roofs.values():
        r["achieved"] = round(r["achieved"], 3)
        r["frac"] = round(r["achieved"] / r["peak"], 4)
        r["avg_ms"] = round(kavg[r["kernel"]], 3)

    phase_names = ["front_extract", "index_build", "index_query", "fp32_scan"]
    if cfg["bf16"]:
        phase_names.append("bf16_scan")
    forms = {
        "index_qps": round(Q / (ph[2] * 1e-3), 1),
        "index_qps_back_to_back": round(Q / (index_b2b_ms * 1e-3), 1) if index_b2b_ms else None,
        "index_qps_with_build": round(Q / ((ph[1] + ph[2]) * 1e-3), 1),
        "fp32_scan_qps": round(Qs / (ph[3] * 1e-3), 1),
        "phase_ms": {k: round(float(v), 3) for k, v in zip(phase_names, ph)},
        "kernel_avg_ms": {k: round(v, 3) for k, v in kavg.items()},
        "fp32_scan_shape": chosen,
        "index_window_trials": window_trials,
        "scan_queries": Qs,
        "index_recall_at_1_pct": round(100 * recall, 3),
        "index_optimal_cost_pct": round(100 * cost_recall, 3),
        "index_acceleration_error_pct": round(ae, 4),
        "rooflines": {k: v for k, v in roofs.items() if k != dom},
    }
    if cfg["bf16"]:
        bi_r, bc_r = res["bi_r"].cpu().numpy(), res["bc_r"].cpu().numpy()
        forms["bf16_scan_qps"] = round(Qs / (ph[4] * 1e-3), 1)
        forms["bf16_vs_fp32_agreement_pct"] = round(
            100 * float(np.mean((bi_r == bi_s) & (bc_r.view(np.uint32) == bc_s.view(np.uint32)))), 3)
        forms["bf16_fallback_queries"] = int(res["fallback"])
        forms["bf16_filter_tiles"] = list(res["tiles"])

    line = {
        "metric": "queries/s at n=1e6,1e8 (SFC index vs GPU brute force), argmin agreement %",
        "value": round(Q / (ms_step * 1e-3), 2),
        "unit": "queries/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32", "data": "synthetic",
        "config": {"workload": cfg["label"],
                   "step": "front + target extraction, index build, index query, float32 scan"
                           + (", bf16 scan" if cfg["bf16"] else "")
                           + " of every front target (value = front targets / step time)",
                   "n": n, "queries": Q, "K": K,
                   "reduced_dim": cfg["D"], "n_curves": cfg["L"], "key_bits": cfg["key_bits"],
                   "window": cfg["window"], "curve": cfg["curve"]},
        "forms": forms,
        "roofline": roofs[dom],
    }

    # the exact k-NN query of Section II.D (k = 80, mu = 256, the paper's
    # parameters) on the same targets, against the float32 scan's answers;
    # Morton indices only, outside the timed steps
    if cfg.get("D") and cfg["curve"] == "morton":
        ixk = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], timing=True,
                           **w.opts)
        for _ in range(2):
            bk, ck = ixk.knn(res["t"], res["m"], k=80, mu=256)
        torch.cuda.synchronize()
        kk = ixk.kernel_times()
        ixk.close()
        k_ms = sum(v[1] / v[0] for v in kk.values())   # one query call
        bk, ck = bk.cpu().numpy(), ck.cpu().numpy()
        okk = bi_s >= 0
        forms["index_knn"] = {
            "k": 80, "mu": 256, "qps": round(Qs / (k_ms * 1e-3), 1),
            "kernel_ms": {k_: round(v[1] / v[0], 3) for k_, v in kk.items()},
            "recall_at_1_pct": round(100 * float(np.mean(bk[okk] == bi_s[okk])), 3),
            "acceleration_error_pct": round(float(np.mean(
                np.sqrt(ck[ok].astype(np.float64)) / np.sqrt(bc_s[ok]) - 1.0)) * 100, 4)}
        log(f"k-NN query: {k_ms:.2f} ms for {Qs} queries")

    # the index rescoring's gather: algorithmic bytes = every candidate's
    # known elements (float32), per query, over one launch
    if cfg.get("D") and "rescore_kernel" in kavg:
        ixc = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], **w.opts)
        fc = native.fill_front(w.mask)
        tc, mc = native.extract_targets(w.vol, w.mask, K, fc)
        _, ncq = ixc.candidates(tc, mc)
        ixc.close()
        known_q = mc.sum(dim=1).double()
        gbytes = float((ncq.double() * known_q).sum().item()) * C * 4
        roofs["rescore_kernel"] = {
            "bound": "hbm", "kernel": "rescore_kernel",
            "achieved": gbytes / (kavg["rescore_kernel"] * 1e-3) / 1e9,
            "peak": PEAK_HBM, "unit": "GB/s", "traffic": None,
            "work_per_launch": f"{gbytes:.4g} bytes = sum over queries of candidates x known "
                               f"elements x 4 (mean {float(ncq.double().mean()):.1f} candidates)"}
        roofs["rescore_kernel"]["achieved"] = round(roofs["rescore_kernel"]["achieved"], 1)
        roofs["rescore_kernel"]["frac"] = round(roofs["rescore_kernel"]["achieved"] / PEAK_HBM, 4)
        roofs["rescore_kernel"]["avg_ms"] = round(kavg["rescore_kernel"], 3)
        forms["rooflines"]["rescore_kernel"] = roofs["rescore_kernel"]
        del fc, tc, mc

    # the brute-force reduced-precision form without an index seed: the
    # two-pass bf16 filter (tile minima, then the tiles that can reach them)
    if cfg["bf16"]:
        ixb = native.Index(w.vol, w.mask, K, timing=True)
        for _ in range(2):
            a_ = ev()
            bu, cu = ixb.query(res["t"], res["m"], "bf16")
            b_ = ev()
            torch.cuda.synchronize()
        kb = ixb.kernel_times()
        p1, p2 = ixb.filter_tiles()
        fbu = ixb.fallbacks()
        ixb.close()
        kd = K ** w.mask_h.ndim
        gemm1 = 2.0 * kd * (C + 2) * n * Qs
        f_ms = sum(v[1] / v[0] for k_, v in kb.items() if k_.startswith("filter_kernel"))
        gemm = gemm1 * (1.0 + (p2 / p1 if p1 else 0.0))
        forms["bf16_two_pass"] = {
            "qps": round(Qs / (a_.elapsed_time(b_) * 1e-3), 1),
            "kernel_ms": {k_: round(v[1] / v[0], 3) for k_, v in kb.items()},
            "filter_tiles": [p1, p2], "fallback_queries": int(fbu),
            "filter_tflops": round(gemm / (f_ms * 1e-3) / 1e12, 1),
            "filter_frac_of_bf16_peak": round(gemm / (f_ms * 1e-3) / 1e12 / PEAK_BF16_MFMA, 4),
            "work": "2 x K^d(C+2) x n x Q x (1 + pass-2 tiles / pass-1 tiles) flop",
            "agreement_with_fp32_pct": round(100 * float(np.mean(
                (bu.cpu().numpy() == bi_s) &
                (cu.cpu().numpy().view(np.uint32) == bc_s.view(np.uint32)))), 3)}
        log(f"bf16 two-pass: {forms['bf16_two_pass']['qps']} q/s")

    # the index forms at the paper's quality acceptance (AE < 1 %)
    if cfg.get("D"):
        fq = native.fill_front(w.mask)
        tq, mq = native.extract_targets(w.vol, w.mask, K, fq)
        forms["index_at_ae_below_1pct"] = quality_point(torch, native, w, tq, mq, ev)
        del fq, tq, mq
        log(f"quality point: {forms['index_at_ae_below_1pct']['windowed'].get('window')} / "
            f"{forms['index_at_ae_below_1pct']['knn'].get('k')}")

    # the L1 cost variant (Section III.K): the float32 scan of the same
    # targets under L1 (second run timed; 2 flops per known element and
    # candidate), outside the timed steps
    ixl = native.Index(w.vol, w.mask, K, norm="l1", timing=True)
    for _ in range(2):
        bl, cl = ixl.query(res["t"], res["m"], "fp32")
    torch.cuda.synchronize()
    kl = ixl.kernel_times()["scan_fp32_kernel"]
    ixl.close()
    l1_ms = kl[1] / kl[0]
    forms["l1_fp32_scan_qps"] = round(Qs / (l1_ms * 1e-3), 1)
    forms["l1_fp32_scan_tflops"] = round(2.0 * known_elems * n / (l1_ms * 1e-3) / 1e12, 2)
    log(f"L1 float32 scan: {l1_ms:.2f} ms for {Qs} queries")

    if args.calib_copy:
        src = torch.ones(1 << 27, dtype=torch.float32, device="cuda:0")
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        log("calibration copy: 536870912 bytes read, 536870912 bytes written")

    if not args.no_cpu_baseline:
        import oracle
        rng = np.random.default_rng(7)
        k = min(args.cpu_sample, Qs)
        sel = np.sort(rng.choice(Qs, k, replace=False))
        t_h = res["t"].cpu().numpy()[sel]
        d_h = oracle.dictionary(w.mask_h, K)
        tc = time.perf_counter()
        ob, oc = oracle.brute(w.vol_h, w.mask_h.shape, K, d_h, t_h, m_h[sel])
        cpu_s = time.perf_counter() - tc
        agree = float(np.mean((ob == bi_s[sel]) & (oc.view(np.uint32) == bc_s[sel].view(np.uint32))))
        line["cpu_baseline"] = {
            "value": round(k / cpu_s, 4), "unit": "queries/s", "cores": 1, "kind": "oracle",
            "cpu_model": cpu_model(), "host_cpus": len(os.sched_getaffinity(0)),
            "sample": f"{k} seeded front queries of the same workload through the oracle's "
                      f"float32 full scan (n={n}), single thread, {cpu_s:.1f}s; index build "
                      f"and index queries excluded (under 0.1% of the oracle's per-query time)"}
        forms["fp32_vs_oracle_agreement_pct"] = round(100 * agree, 2)
        # the same oracle with the query list split over the host cores (ctypes
        # releases the GIL, so the threads run the C scan in parallel)
        cores = min(16, len(os.sched_getaffinity(0)))
        k2 = min(12 * cores, Qs)
        sel2 = np.sort(np.random.default_rng(8).choice(Qs, k2, replace=False))
        t2_h, m2_h = res["t"].cpu().numpy()[sel2], m_h[sel2]
        parts = np.array_split(np.arange(k2), cores)
        from concurrent.futures import ThreadPoolExecutor
        tc = time.perf_counter()
        with ThreadPoolExecutor(cores) as ex:
            outs = list(ex.map(lambda ix: oracle.brute(w.vol_h, w.mask_h.shape, K, d_h, t2_h[ix],
                                                       m2_h[ix]), parts))
        par_s = time.perf_counter() - tc
        ob2 = np.concatenate([o[0] for o in outs])
        oc2 = np.concatenate([o[1] for o in outs])
        agree2 = float(np.mean((ob2 == bi_s[sel2]) & (oc2.view(np.uint32) == bc_s[sel2].view(np.uint32))))
        forms["cpu_oracle_all_cores"] = {
            "value": round(k2 / par_s, 3), "unit": "queries/s", "cores": cores,
            "sample": f"{k2} seeded front queries split over {cores} threads, {par_s:.1f}s",
            "agreement_with_fp32_scan_pct": round(100 * agree2, 2)}
        log(f"oracle on {cores} threads: {k2} queries in {par_s:.1f}s")
        # the L1 scan's answers against the oracle's L1 scan on 4 of them
        s4 = sel[:4]
        ob1, oc1 = oracle.brute(w.vol_h, w.mask_h.shape, K, d_h, t_h[:4], m_h[s4], norm="l1")
        bl_h, cl_h = bl.cpu().numpy()[s4], cl.cpu().numpy()[s4]
        forms["l1_vs_oracle_agreement_pct"] = round(
            100 * float(np.mean((ob1 == bl_h) & (oc1.view(np.uint32) == cl_h.view(np.uint32)))), 2)

    if args.workload == "config2" and not args.no_inpaint:
        del res
        torch.cuda.empty_cache()
        line["inpaint"] = inpaint_pass(torch, native, synth, ("config1", "config2", "config3"))
        res = None
    if args.workload == "config2" and not args.no_n1e8:
        del w, res
        torch.cuda.empty_cache()
        line["n1e8"] = large_pass(torch, native, synth, ev)
    if args.workload == "config2" and not args.no_batch:
        torch.cuda.empty_cache()
        line["batch"] = batch_pass(torch, native, synth, ev, 16, (256, 1024), 3, 1)
    print(json.dumps(line), flush=True)


KNN_KS = (4, 8, 12, 16, 24, 32, 48, 64, 80, 96, 128, 160, 192, 256)


def _accel_error(ci, cs):
    """Section III.C's acceleration error (mean of sqrt(cost_index /
    cost_scan) - 1 over targets with a nonzero scan cost), as a fraction."""
    ok = cs > 0
    return float(np.mean(np.sqrt(ci[ok].astype(np.float64)) / np.sqrt(cs[ok].astype(np.float64))
                         - 1.0)) if ok.any() else 0.0


def quality_point(torch, native, w, t, m, ev, sample=1024):
    """Section III.D accepts an acceleration error below 1 %. On a seeded
    sample of front targets: the smallest window W of the windowed query
    (sfc_autotune_window with a 1 % target) and the smallest k of the exact
    k-NN query (mu = 256) whose error is below 1 %, each with its query rate
    over every front target (second run timed)."""
    cfg, K = w.cfg, w.K
    Q = int(m.shape[0])
    k = min(sample, Q)
    sel = torch.from_numpy(np.sort(np.random.default_rng(11).choice(Q, k, replace=False))).cuda()
    ts, ms = t[sel].contiguous(), m[sel].contiguous()
    out = {"sample": k, "accel_error_limit_pct": 1.0}
    ix = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], **w.opts)
    ref_i, ref_c = (a.cpu().numpy() for a in ix.query(ts, ms, "fp32"))
    W, trials = ix.autotune_window(ts, ms, 0.0, 0.01)
    hit = next((x for x in trials if x["accel_error"] < 0.01), None)
    win = {"trials": [{"window": x["window"], "recall_pct": round(100 * x["recall"], 2),
                       "accel_error_pct": round(100 * x["accel_error"], 4)} for x in trials]}
    if hit is not None:
        for _ in range(2):
            a = ev()
            ix.query(t, m, "index")
            b = ev()
            torch.cuda.synchronize()
        ms_ = a.elapsed_time(b)
        win.update(reached=True, window=W, candidates_per_query=W * cfg["L"],
                   recall_pct=round(100 * hit["recall"], 2),
                   accel_error_pct=round(100 * hit["accel_error"], 4),
                   qps=round(Q / (ms_ * 1e-3), 1))
    else:
        last = trials[-1]
        win.update(reached=False, largest_window=last["window"],
                   accel_error_pct_at_largest=round(100 * last["accel_error"], 4))
    out["windowed"] = win
    knn = {"mu": 256, "trials": []}
    if cfg["curve"] == "morton":
        for kk in KNN_KS:
            bk, ck = (a.cpu().numpy() for a in ix.knn(ts, ms, k=kk, mu=256))
            ae = _accel_error(ck, ref_c)
            knn["trials"].append({"k": kk, "recall_pct": round(100 * float(np.mean(bk == ref_i)), 2),
                                  "accel_error_pct": round(100 * ae, 4)})
            if ae < 0.01:
                for _ in range(2):
                    a = ev()
                    ix.knn(t, m, k=kk, mu=256)
                    b = ev()
                    torch.cuda.synchronize()
                ms_ = a.elapsed_time(b)
                knn.update(reached=True, k=kk, recall_pct=knn["trials"][-1]["recall_pct"],
                           accel_error_pct=round(100 * ae, 4), qps=round(Q / (ms_ * 1e-3), 1))
                break
        else:
            knn.update(reached=False)
    out["knn"] = knn
    ix.close()
    return out


def inpaint_pass(torch, native, synth, names=("config1", "config2")):
    """Whole inpainting runs (Section I's fill loop in Criminisi order, the
    analogue of the paper's Table 2 on synthetic images): the device-resident
    loop with the float32 full scan and with the SFC index (its build timed
    apart), each on a fresh copy of the image."""
    out = {}
    for name in names:
        cfg = WORKLOADS[name]
        d = getattr(synth, cfg["gen"])()
        vol0 = torch.from_numpy(d["volume"]).cuda()
        mask0 = torch.from_numpy(d["mask"]).cuda()
        K = cfg["K"]
        row = {"unknown_voxels": int((d["mask"] == 0).sum()), "K": K}
        for mode in ("fp32", "index"):
            vol, mask = vol0.clone(), mask0.clone()
            torch.cuda.synchronize()
            ix = None
            build_ms = 0.0
            if mode == "index":
                tb = time.perf_counter()
                ix = native.Index(vol, mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"],
                                  key_bits=cfg["key_bits"], window=cfg["window"], curve=cfg["curve"])
                torch.cuda.synchronize()
                build_ms = 1e3 * (time.perf_counter() - tb)
            tl = time.perf_counter()
            it, _ = native.inpaint(vol, mask, K, order="criminisi", mode=mode, index=ix)
            torch.cuda.synchronize()
            loop_ms = 1e3 * (time.perf_counter() - tl)
            if ix is not None:
                ix.close()
            row[mode] = {"iterations": it, "loop_ms": round(loop_ms, 1),
                         "ms_per_iteration": round(loop_ms / max(it, 1), 4)}
            if mode == "index":
                row[mode]["index_build_ms"] = round(build_ms, 1)
                row[mode]["total_ms"] = round(loop_ms + build_ms, 1)
            log(f"inpaint {name} {mode}: {it} iterations in {loop_ms:.0f} ms")
        row["index_speedup_over_fp32_scan"] = round(row["fp32"]["loop_ms"] / row["index"]["total_ms"], 2)
        out[name] = row
        del vol0, mask0
        torch.cuda.empty_cache()
    return out


def batch_pass(torch, native, synth, ev, n_images, sides, steps, warmup):
    """Uneven images answered together: every front target of every image by
    one persistent float32-scan launch, replayed from a HIP graph (tile-shape
    set from the batch autotuner). Two images are checked against the
    single-image scan."""
    t0 = time.time()
    imgs = synth.config5(n_images=n_images, side_range=sides)
    log(f"generated {n_images} images in {time.time() - t0:.1f}s")
    K = 9
    vols = [torch.from_numpy(d["volume"]).cuda() for d in imgs]
    masks = [torch.from_numpy(d["mask"]).cuda() for d in imgs]
    ts, ms, counts = [], [], []
    for v, m in zip(vols, masks):
        f = native.fill_front(m)
        t, mm = native.extract_targets(v, m, K, f)
        ts.append(t.reshape(-1))
        ms.append(mm)
        counts.append(int(f.numel()))
    t = torch.cat(ts).contiguous()
    m = torch.cat(ms).contiguous()
    Q = sum(counts)
    b = native.Batch(vols, masks, K)
    out = (torch.empty(Q, dtype=torch.int64, device="cuda"),
           torch.empty(Q, dtype=torch.float32, device="cuda"))
    shape = b.autotune(t, m, counts, out)
    for _ in range(warmup):
        b.query(t, m, counts, out)
    torch.cuda.synchronize()
    a = ev()
    for _ in range(steps):
        b.query(t, m, counts, out)
    e = ev()
    torch.cuda.synchronize()
    ms_rep = a.elapsed_time(e) / steps
    st = b.stats()
    # the first two images against the single-image float32 scan
    agree, toff, qoff = [], 0, 0
    for i, d in enumerate(imgs[:2]):
        C = d["volume"].shape[-1]
        q = counts[i]
        ix = native.Index(vols[i], masks[i], K)
        bi, bc = ix.query(t[toff: toff + q * K * K * C].reshape(q, K * K, C).contiguous(),
                          m[qoff: qoff + q].contiguous(), "fp32")
        agree.append(bool(torch.equal(bi, out[0][qoff: qoff + q]) and
                          torch.equal(bc.view(torch.int32), out[1][qoff: qoff + q].view(torch.int32))))
        ix.close()
        toff += q * K * K * C
        qoff += q
    b.close()
    return {"images": n_images, "sides": list(sides), "queries": Q,
            "pixels": int(sum(x.numel() for x in masks)),
            "ms_per_replay": round(ms_rep, 3), "qps": round(Q / (ms_rep * 1e-3), 1),
            "work_items": st["work_items"], "graph_replays": st["graph_replays"],
            "shape_set": shape, "equals_single_image_scan": all(agree)}


def large_pass(torch, native, synth, ev):
    """One pass over the 512^3 volume: build, index query of the whole front,
    float32 scan of a seeded 4096-target sample (each query form timed on its
    second run)."""
    w = Workload("config4", torch, native, synth)
    cfg, K = w.cfg, w.K
    f = native.fill_front(w.mask)
    t, m = native.extract_targets(w.vol, w.mask, K, f)
    e0 = ev()
    ix = native.Index(w.vol, w.mask, K, reduced_dim=cfg["D"], n_curves=cfg["L"], timing=True,
                      **w.opts)
    e1 = ev()
    torch.cuda.synchronize()
    build_ms = e0.elapsed_time(e1)
    log(f"n~1.25e8: index built in {build_ms:.0f} ms")
    ix.set_timing(False)   # the index query's own time, without timing events
    for _ in range(2):
        a = ev()
        bi_x, bc_x = ix.query(t, m, "index")
        b = ev()
        torch.cuda.synchronize()
    idx_ms = a.elapsed_time(b)
    ix.set_timing(True)
    ts, ms = t[w.sel].contiguous(), m[w.sel].contiguous()
    # the float32 scan's tile shape, autotuned on the first 512 sampled targets
    shape = ix.autotune(ts[:512].contiguous(), ms[:512].contiguous())
    log(f"n~1.25e8: autotuned float32-scan shape {shape}")
    for _ in range(2):
        a = ev()
        bi_s, bc_s = ix.query(ts, ms, "fp32")
        b = ev()
        torch.cuda.synchronize()
    scan_ms = a.elapsed_time(b)
    kt = ix.kernel_times()
    n = ix.info.n
    # the exact k-NN query of Section II.D on the same sample (k = 80, mu = 256)
    for _ in range(2):
        bk, ck = ix.knn(ts, ms, k=80, mu=256)
    torch.cuda.synchronize()
    kk = ix.kernel_times()
    knn_ms = sum(v[1] / v[0] for v in kk.values())   # one query call
    ix.close()
    quality = quality_point(torch, native, w, t, m, ev)
    bx, cx = bi_x[w.sel].cpu().numpy(), bc_x[w.sel].cpu().numpy()
    bs, cs = bi_s.cpu().numpy(), bc_s.cpu().numpy()
    ok = cs > 0
    known = float(ms.sum().item())
    scan_tf = 3.0 * known * n / (kt["scan_fp32_kernel"][1] / kt["scan_fp32_kernel"][0] * 1e-3) / 1e12
    out = {"workload": cfg["label"], "n": n, "queries": w.Q, "scan_queries": int(ms.shape[0]),
           "index_build_ms": round(build_ms, 1),
           "index_qps": round(w.Q / (idx_ms * 1e-3), 1),
           "fp32_scan_qps": round(ms.shape[0] / (scan_ms * 1e-3), 2),
           "fp32_scan_tflops": round(scan_tf, 2),
           "fp32_scan_frac_of_fp32_peak": round(scan_tf / PEAK_FP32_VALU, 4),
           "fp32_scan_shape": shape,
           "index_recall_at_1_pct": round(100 * float(np.mean(bx == bs)), 3),
           "index_optimal_cost_pct": round(100 * float(np.mean(cx.view(np.uint32) == cs.view(np.uint32))), 3),
           "index_acceleration_error_pct": round(
               float(np.mean(np.sqrt(cx[ok].astype(np.float64)) / np.sqrt(cs[ok]) - 1)) * 100, 4),
           "index_cost_never_below_scan": bool(np.all(cx >= cs)),
           "index_knn": {"k": 80, "mu": 256, "qps": round(ms.shape[0] / (knn_ms * 1e-3), 1),
                         "recall_at_1_pct": round(100 * float(np.mean(bk.cpu().numpy() == bs)), 3),
                         "acceleration_error_pct": round(float(np.mean(
                             np.sqrt(ck.cpu().numpy()[ok].astype(np.float64)) / np.sqrt(cs[ok])
                             - 1)) * 100, 4)},
           "index_at_ae_below_1pct": quality}
    del w, t, m, ts, ms
    torch.cuda.empty_cache()
    return out


if __name__ == "__main__":
    main()
