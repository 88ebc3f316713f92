"""Benchmark: batched chemical source-term throughput on one MI355X.

A step is one evaluation of the whole source term (concentrations, Gibbs and
Arrhenius layers, rates of progress, production rates; Barwey & Raman,
Sec. 2) over one batch of synthetic cells already resident in HBM.  The
default workload is the 53-species / 325-reaction synthetic mechanism over
2^20 cells with FP32 states (the throughput target size), FP32 path.

Prints one JSON line.  Extra keys: the FP64 path on the same workload,
per-step latency percentiles, the FP32-vs-FP64 difference, the 65,536-cell
precision configuration, the roofline of the kernel, a saturation curve over
batch size, the Jacobian and VJP, the serving loop, the 111/784 mechanism,
and the CPU oracle on all host cores and on one.
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

from paper_2008_08483_amd import roofline, synth  # noqa: E402

TRAFFIC_FILE = os.path.join(ROOT, "profiles", "traffic_source_f32_53x325_1M.json")


def kernel_source_hash(src=None) -> str:
    """Identity of the FP32 source-term kernel the workload runs: the hash of
    the generated source text (compiled kernels), else of the table
    kernels' sources."""
    h = hashlib.sha256()
    if src is None:
        src = synth.workload("c1_full", n_cells=1)[0]
    from paper_2008_08483_amd import annkin
    try:
        text = annkin.jit_source(src, "fp32")
    except Exception:  # pragma: no cover - library missing: fall back to files
        text = None
    if text is not None and src.n_species <= 102:
        h.update(text.encode())
    else:
        for f in ("source_kernels.hip", "ak_device.h", "ak_math.h"):
            with open(os.path.join(ROOT, "paper_2008_08483_amd", "csrc", f), "rb") as fh:
                h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch from committed rocprofv3 counter runs, or None
    if absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_hash") != kernel_source_hash():
        return None
    return t.get("bytes_per_launch")


def accuracy(torch, annkin, mech, src, T, P, Y, n=4096):
    """Error of both paths against the oracle on the first n cells: FP32 path
    against the double oracle on the exact FP32 inputs, FP64 path against the
    extended-precision oracle (metrics M1 = |d omega|/S, M2 = |d omega|/N over
    entries with N >= S/kappa, M3 = |d omega|/|omega| over |omega| >= 1e-3 S)."""
    import oracle
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from metrics import grade
    T, P, Y = (np.asarray(a)[..., :n] for a in (T, P, Y))
    out = {}
    for name, dt, prec, kappa in (("fp32", np.float32, "f64", 1e4), ("fp64", np.float64, "ld", 10.0)):
        Ti, Pi, Yi = (np.ascontiguousarray(a.astype(dt)) for a in (T, P, Y))
        tdt = torch.float32 if dt == np.float32 else torch.float64
        om = annkin.eval_source(mech, *(torch.tensor(a, dtype=tdt, device="cuda") for a in (Ti, Pi, Yi)))
        torch.cuda.synchronize()
        om = om.cpu().numpy().astype(np.float64)
        ref, S, N = oracle.source(src, *(a.astype(np.float64) for a in (Ti, Pi, Yi)),
                                  precision=prec, scales=True)
        g = grade(om, ref, S, N, kappa_max=kappa, s_floor=1e-30 if dt == np.float32 else 0.0)
        out[name] = {k: g[k] for k in ("m1_max", "m1_median", "m2_max", "m3_median", "m3_p99",
                                       "nonfinite")}
    out["sample"] = f"first {n} cells of the workload; FP32 vs the double oracle, FP64 vs the " \
                    "extended-precision oracle"
    return out


def time_path(torch, annkin, mech, T, P, Y, steps, warmup):
    """Whole-step wall time (barrier + sync around K steps) and per-launch
    kernel durations from HIP events on the launch stream."""
    out = torch.empty_like(Y)
    for _ in range(warmup):
        annkin.eval_source(mech, T, P, Y, out=out)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    t0 = time.perf_counter()
    for i in range(steps):
        ev[i][0].record(stream)
        annkin.eval_source(mech, T, P, Y, out=out)
        ev[i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = np.array([a.elapsed_time(b) for a, b in ev])
    return wall, ms, out


def cpu_baseline(src, T, P, Y, target_s=12.0):
    """The oracle (plain C, double, OpenMP over cells) on the host cores, on
    a bounded sample of the same workload."""
    import oracle
    cores = len(os.sched_getaffinity(0))
    env = os.environ.get("OMP_NUM_THREADS")
    if env and env.isdigit():
        cores = min(cores, int(env))
    T64, P64, Y64 = (np.asarray(a, np.float64) for a in (T, P, Y))
    n0 = min(256 * cores, T64.shape[0])
    t0 = time.perf_counter()
    oracle.source(src, T64[:n0], P64[:n0], Y64[:, :n0], n_threads=cores)
    dt0 = time.perf_counter() - t0
    n = int(min(T64.shape[0], max(n0, n0 * target_s / max(dt0, 1e-3))))
    t0 = time.perf_counter()
    oracle.source(src, T64[:n], P64[:n], Y64[:, :n], n_threads=cores)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "cells/s", "cores": cores, "kind": "oracle",
            "sample": f"first {n} cells of the workload, double precision, "
                      f"{cores} OpenMP threads, {dt:.1f} s"}


def cpu_single_core(src, T, P, Y, target_s=8.0):
    """The same oracle on one host core (the paper's one-rank baseline)."""
    import oracle
    T64, P64, Y64 = (np.asarray(a, np.float64) for a in (T, P, Y))
    n0 = min(512, T64.shape[0])
    t0 = time.perf_counter()
    oracle.source(src, T64[:n0], P64[:n0], Y64[:, :n0], n_threads=1)
    dt0 = time.perf_counter() - t0
    n = int(min(T64.shape[0], max(n0, n0 * target_s / max(dt0, 1e-3))))
    t0 = time.perf_counter()
    oracle.source(src, T64[:n], P64[:n], Y64[:, :n], n_threads=1)
    dt = time.perf_counter() - t0
    return {"value": n / dt, "unit": "cells/s", "cores": 1, "kind": "oracle",
            "sample": f"first {n} cells of the workload, double precision, 1 thread, "
                      f"{dt:.1f} s"}


def kernel_ms(torch, annkin, mech, T, P, Y, reps=20, warmup=3):
    """Median kernel time (HIP events on the launch stream) of eval_source."""
    out = torch.empty((Y.shape[0], T.shape[0]), dtype=T.dtype, device="cuda")
    for _ in range(warmup):
        annkin.eval_source(mech, T, P, Y, out=out)
    stream = torch.cuda.current_stream()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(reps)]
    for a, b in ev:
        a.record(stream)
        annkin.eval_source(mech, T, P, Y, out=out)
        b.record(stream)
    torch.cuda.synchronize()
    return float(np.median([a.elapsed_time(b) for a, b in ev]))


def saturation(torch, annkin, mech, T, P, Y):
    """FP32 throughput against batch size: the first n cells of the
    workload, n = 2^6 .. 2^20 (the analogue of the paper's cells-per-rank
    sweep, Sec. 3.2)."""
    out = []
    for e in range(6, 21, 2):
        n = 1 << e
        if n > T.shape[0]:
            break
        ms = kernel_ms(torch, annkin, mech, T[:n], P[:n], Y[:, :n])
        out.append({"n_cells": n, "kernel_ms": ms, "cells_per_s": n / (ms * 1e-3)})
    return out


def c2_bench(torch, annkin):
    """The 111-species / 784-reaction mechanism over 2^20 cells, both paths."""
    src, T, P, Y = synth.workload("c2", dtype=np.float32)
    mech = annkin.Mechanism(src)
    n = T.shape[0]
    res = {"workload": f"{src.n_species}sp/{src.n_reactions}rxn synthetic mechanism x {n} "
                       "cells"}
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        Tt, Pt, Yt = (torch.tensor(a, device="cuda").to(dt) for a in (T, P, Y))
        ms = kernel_ms(torch, annkin, mech, Tt, Pt, Yt, reps=10)
        res[name] = {"kernel_ms": ms, "cells_per_s": n / (ms * 1e-3)}
        del Tt, Pt, Yt
    slots = roofline.method_slots(src.nu_f, src.nu_r)
    res["roofline_frac_fp32"] = slots * n / (res["fp32"]["kernel_ms"] * 1e-3) / \
        roofline.PEAK_VALU_SLOTS
    mech.close()
    return res


def pdep_bench(torch, annkin, T32, P32, Y32, T, P, Y):
    """The 53/325 mechanism with 20 % of its reactions pressure dependent
    (third-body, Lindemann and Troe falloff; Sec. 2.4) on the same 2^20
    states, both paths, and its error against the oracle."""
    src = synth.with_pressure_dependence(synth.make_mechanism(53, 325), frac=0.2)
    mech = annkin.Mechanism(src)
    n = T32.shape[0]
    counts = np.bincount(src.rtype, minlength=4)
    res = {"workload": f"{src.n_species}sp/{src.n_reactions}rxn synthetic mechanism, "
                       f"{int(counts[1])} third-body, {int(counts[2])} Lindemann, "
                       f"{int(counts[3])} Troe reactions, x {n} cells"}
    for name, dt in (("fp32", torch.float32), ("fp64", torch.float64)):
        Tt, Pt, Yt = (a.to(dt) for a in (T32, P32, Y32))
        ms = kernel_ms(torch, annkin, mech, Tt, Pt, Yt, reps=10)
        res[name] = {"kernel_ms": ms, "cells_per_s": n / (ms * 1e-3)}
        del Tt, Pt, Yt
    res["accuracy"] = accuracy(torch, annkin, mech, src, T, P, Y, n=2048)
    mech.close()
    return res


def _serving_pools(torch, annkin, mechs, nmax):
    """Page-locked host states per mechanism (requests use the first n cells,
    leading dimension nmax) and a shared output scratch per mechanism."""
    pools = []
    for i, src in enumerate(mechs):
        T, P, Y = synth.make_states(src, nmax, 3000 + i, (800.0, 2800.0), (1.0, 20.0), 0.3,
                                    dtype=np.float32)
        pin = lambda a: torch.from_numpy(np.ascontiguousarray(a)).pin_memory()
        pools.append((pin(T), pin(P), pin(Y),
                      torch.zeros((src.n_species, nmax), dtype=torch.float32).pin_memory()))
    return pools


def _run_trace(annkin, srv, dev_mechs, pools, arrivals, sizes, which, warmup):
    """Open-loop replay: submit request i at arrivals[i] (seconds from start);
    a second thread waits for and frees completed requests.  Statistics are
    reset after `warmup` requests have completed."""
    import queue
    import threading
    q = queue.Queue()
    done = [0]

    def reaper():
        while True:
            r = q.get()
            if r is None:
                return
            r.wait(120.0)
            r.free()
            done[0] += 1
            if done[0] == warmup:
                srv.reset_stats()

    th = threading.Thread(target=reaper)
    th.start()
    t0 = time.perf_counter()
    for i in range(len(sizes)):
        delay = arrivals[i] - (time.perf_counter() - t0)
        if delay > 2e-3:
            time.sleep(delay - 1e-3)
        while time.perf_counter() - t0 < arrivals[i]:
            pass
        k, n = int(which[i]), int(sizes[i])
        T, P, Y, O = pools[k]
        q.put(srv.submit(dev_mechs[k], T[:n], P[:n], Y[:, :n], O[:, :n]))
    q.put(None)
    th.join()
    return srv.stats()


def serving_bench(torch, annkin, n_req=10000, warmup=500, trials=3):
    """Serving configuration: requests of log-uniform [64, 65536] cells, half
    on the 9/21 and half on the 53/325 mechanism (both resident), FP32.
    Capacity of the one-launch-per-request form measured closed-loop, then
    both forms replay one seeded Poisson trace at 0.8x that capacity, three
    times each, interleaved."""
    srcs = [synth.make_mechanism(9, 21), synth.make_mechanism(53, 325)]
    dev = [annkin.Mechanism(s) for s in srcs]
    nmax = 65536
    pools = _serving_pools(torch, annkin, srcs, nmax)
    _, sizes, which = synth.make_trace(n_req + warmup, 1.0, seed=2000)
    sizes = np.minimum(sizes, nmax)
    # capacity: closed loop, 8 outstanding, one launch per request
    srv = annkin.Server(batching=False, max_inflight=3)
    outstanding, t0, cells = [], time.perf_counter(), 0
    m = min(3000, len(sizes))
    for i in range(m):
        k, n = int(which[i]), int(sizes[i])
        T, P, Y, O = pools[k]
        outstanding.append(srv.submit(dev[k], T[:n], P[:n], Y[:, :n], O[:, :n]))
        cells += n
        if len(outstanding) >= 8:
            r = outstanding.pop(0)
            r.wait(120.0)
            r.free()
    for r in outstanding:
        r.wait(120.0)
        r.free()
    cap_s = m / (time.perf_counter() - t0)
    srv.close()
    rate = 0.8 * cap_s
    arrivals, _, _ = synth.make_trace(n_req + warmup, rate, seed=2000)
    out = {"workload": "requests of log-uniform [64, 65536] cells, 50/50 9sp/21rxn and "
                       "53sp/325rxn mechanisms, FP32, Poisson arrivals",
           "capacity_one_launch_req_per_s": cap_s, "offered_req_per_s": rate,
           "requests": n_req, "warmup_requests": warmup, "trials": trials,
           "note": "p50/p99 are medians over trials of the same seeded trace, the two "
                   "modes interleaved"}
    runs = {"one_launch_per_request": [], "continuous_batching": []}
    for _ in range(trials):
        for name, batching in (("one_launch_per_request", False), ("continuous_batching", True)):
            srv = annkin.Server(batching=batching, max_inflight=3, arena_bytes=1 << 30)
            st = _run_trace(annkin, srv, dev, pools, arrivals, sizes, which, warmup)
            srv.close()
            runs[name].append(st)
    for name, sts in runs.items():
        med = lambda k: float(np.median([st[k] for st in sts]))
        out[name] = {"p50_ms": med("p50_ms"), "p99_ms": med("p99_ms"), "mean_ms": med("mean_ms"),
                     "cells_per_s": med("cells_per_s"),
                     "p50_ms_trials": [st["p50_ms"] for st in sts],
                     "p99_ms_trials": [st["p99_ms"] for st in sts],
                     "completed": sts[-1]["completed"], "batches": sts[-1]["batches"],
                     "launches": sts[-1]["launches"]}
    for d in dev:
        d.close()
    return out


def deriv_bench(torch, annkin, steps=10):
    """Differentiation configuration: 53/325 mechanism x 65,536 cells; the
    dense 54 x 54 per-cell Jacobian (compiled kernel in both output layouts,
    and the table-driven kernel beside it) and the VJP, FP64 and FP32 states.
    The Jacobian's roofline is its HBM write (n (NS+1)^2 elements)."""
    src, T, P, Y = synth.workload("c4")
    mech = annkin.Mechanism(src)
    n, nv = T.shape[0], src.n_species + 1
    out = {"workload": f"{src.n_species}sp/{src.n_reactions}rxn synthetic mechanism x {n} cells",
           "jacobian_kernel": "compiled" if mech.compiled_jacobian(torch.float64) else "table"}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    for name, dt in (("fp64", torch.float64), ("fp32", torch.float32)):
        Tt, Pt, Yt = (torch.tensor(a, dtype=dt, device="cuda") for a in (T, P, Y))
        J = torch.empty((n, nv, nv), dtype=dt, device="cuda")
        g = torch.randn((src.n_species, n), dtype=dt, device="cuda")
        res = {}
        es = 8 if dt == torch.float64 else 4
        jbytes = n * nv * nv * es
        legs = [("jacobian", lambda: annkin.eval_jacobian(mech, Tt, Pt, Yt, out=J)),
                ("vjp", lambda: annkin.eval_vjp(mech, Tt, Pt, Yt, g))]
        if mech.compiled_jacobian(dt):
            Ji = torch.empty((nv, nv, n), dtype=dt, device="cuda")
            legs.append(("jacobian_interleaved",
                         lambda: annkin.eval_jacobian_interleaved(mech, Tt, Pt, Yt, out=Ji)))
        for what, fn in legs:
            ms = timed(fn)
            res[what + "_ms"] = ms
            res[what + "_per_s"] = n / (ms * 1e-3)
            if what.startswith("jacobian"):
                res[what + "_write_GBps"] = jbytes / (ms * 1e-3) / 1e9
                res[what + "_write_frac_of_hbm"] = jbytes / (ms * 1e-3) / roofline.PEAK_HBM
        if mech.compiled_jacobian(dt):
            # bitwise: repeated calls and the two layouts
            J2 = annkin.eval_jacobian(mech, Tt, Pt, Yt)
            torch.cuda.synchronize()
            res["jacobian_bitwise_repeat"] = bool(torch.equal(J, J2))
            res["jacobian_layouts_bitwise_equal"] = bool(torch.equal(J.permute(1, 2, 0), Ji))
            del J2, Ji
            os.environ["AK_JIT_JACOBIAN"] = "0"
            try:
                res["jacobian_table_kernel_ms"] = timed(
                    lambda: annkin.eval_jacobian(mech, Tt, Pt, Yt, out=J))
            finally:
                del os.environ["AK_JIT_JACOBIAN"]
        res["jacobian_roofline_ms"] = jbytes / roofline.PEAK_HBM * 1e3
        # one linearly implicit Euler step of the 0-D reactor (Jacobian,
        # source term, then one workgroup per cell solving its 54 x 54
        # system), on copies of the states; dt far past explicit stability
        T2, Y2 = Tt.clone(), Yt.clone()
        res["implicit_step_ms"] = timed(
            lambda: annkin.integrate_implicit(mech, T2, Pt, Y2, 1e-12, 1))
        res["implicit_step_cells_per_s"] = n / (res["implicit_step_ms"] * 1e-3)
        del T2, Y2
        out[name] = res
        del Tt, Pt, Yt, J, g
    mech.close()
    return out


def prod_bench(torch, annkin, steps=20):
    """The stoichiometric contraction omega = nu r from given FP32 rates of
    progress on the matrix cores in split bfloat16 (ak_eval_production),
    53/325 x 2^20 and 150/600 x 2^19 cells.  It is HBM-bound: the
    algorithmic traffic is (N_R + N_S) x 4 bytes per cell.  Beside it, the
    same product as a dense FP32 library GEMM (torch.matmul) for context,
    and the error of the sampled result against nu r in float64 relative to
    sum |nu| |r| (the FP32 dot-product error, about 2^-24 per term)."""
    rows = {}
    for ns, nr, n in ((53, 325, 1 << 20), (150, 600, 1 << 19)):
        src = synth.make_mechanism(ns, nr)
        mech = annkin.Mechanism(src)
        g = torch.Generator(device="cuda").manual_seed(1)
        r = torch.randn((nr, n), generator=g, device="cuda", dtype=torch.float32)
        out = torch.empty((ns, n), dtype=torch.float32, device="cuda")
        nu = torch.tensor((src.nu_r.astype(np.float32) - src.nu_f.astype(np.float32)).T,
                          device="cuda").contiguous()

        def timed(fn):
            fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                fn()
            e1.record()
            torch.cuda.synchronize()
            return e0.elapsed_time(e1) / steps

        ms = timed(lambda: annkin.eval_production(mech, r, out=out))
        ms_mm = timed(lambda: torch.matmul(nu, r))
        byt = (nr + ns) * 4 * n
        idx = torch.arange(0, n, 257, device="cuda")
        rs = r[:, idx].double()
        want = nu.double() @ rs
        err = ((out[:, idx].double() - want).abs() / (nu.double().abs() @ rs.abs())
               .clamp_min(1e-300)).max().item()
        rows[f"{ns}x{nr}"] = {
            "n_cells": n, "ms": ms, "cells_per_s": n / (ms * 1e-3),
            "hbm_GBps": byt / (ms * 1e-3) / 1e9, "hbm_frac": byt / (ms * 1e-3) / roofline.PEAK_HBM,
            "torch_fp32_matmul_ms": ms_mm, "max_err_rel_to_sum_abs": err}
        del r, out
        mech.close()
    return rows


def kc_bench(torch, annkin, steps=20, train=True):
    """The trained ln K_c network of Sec. 2.3 (Architecture 2) against the
    exact Gibbs and stoichiometric layers, at the paper's N_C = 10^5 (its
    Fig. 10 point): the time of each to write ln K_c [N_R, N_C] for the
    9/21 and 53/325 mechanisms over N_L in {1, 2, 3} x N_H in
    {8, 16, 32, 64}, FP32 and FP64, and the ratio exact / network.  Both
    write N_R N_C elements, their HBM bound.  With ``train``, LF (1/8) and HF
    (3/32) networks are fitted on the GPU to 10^6 (T, ln K_c) pairs of the
    53/325 mechanism (T ~ U[300, 3000] K, ln K_c from ak_eval_lnkc) and the
    source term with each network in place of ln K_c is compared with the
    exact compiled source term on the differentiation states (53/325 x 65,536)."""
    from paper_2008_08483_amd import kcnet
    n = 100_000
    rng = np.random.default_rng(77)
    out = {"n_cells": n, "definition": "speedup = exact ln K_c time / network time "
           "(both write ln K_c [N_R, N_C]); hbm_frac = (N_R + 1) N_C s / time / 8 TB/s"}

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / steps

    grid = [(l, h) for l in (1, 2, 3) for h in (8, 16, 32, 64)]
    for ns, nr in ((9, 21), (53, 325)):
        src = synth.make_mechanism(ns, nr)
        mech = annkin.Mechanism(src)
        rows = {}
        for pname, dt, es in (("fp32", torch.float32, 4), ("fp64", torch.float64, 8)):
            Tt = torch.tensor(rng.uniform(800.0, 2800.0, n), dtype=dt, device="cuda")
            K = torch.empty((nr, n), dtype=dt, device="cuda")
            bytes_ = (nr + 1) * n * es
            t_ex = timed(lambda: annkin.eval_lnkc(mech, Tt, out=K))
            r = {"exact_ms": t_ex, "exact_hbm_frac": bytes_ / (t_ex * 1e-3) / roofline.PEAK_HBM}
            for l, h in grid:
                net = annkin.KcNet(kcnet.random_weights(l, h, nr, seed=l * 100 + h))
                t = timed(lambda: annkin.eval_lnkc_net(net, Tt, out=K))
                r[f"{l}/{h}"] = {"ms": t, "speedup": t_ex / t,
                                 "hbm_frac": bytes_ / (t * 1e-3) / roofline.PEAK_HBM,
                                 "flops_TF": 2.0 * n * (h + (l - 1) * h * h + h * nr) /
                                             (t * 1e-3) / 1e12}
                net.close()
            rows[pname] = r
            del Tt, K
        out[f"{ns}x{nr}"] = rows
        mech.close()
    if not train:
        return out
    src, T, P, Y = synth.workload("c4")
    mech = annkin.Mechanism(src)
    t0 = time.perf_counter()
    Ttr, Ktr = kcnet.training_set(mech, n=1_000_000, T_range=(300.0, 3000.0), seed=5)
    out["training_set_s"] = time.perf_counter() - t0
    Tt, Pt, Yt = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in (T, P, Y))
    ex = annkin.eval_source(mech, Tt, Pt, Yt)
    Kst = annkin.eval_lnkc(mech, Tt)
    big = ex.abs() >= 1e-6 * ex.abs().max()
    Tv = torch.tensor(rng.uniform(300.0, 3000.0, 200_000), dtype=torch.float64, device="cuda")
    Kv = annkin.eval_lnkc(mech, Tv)
    t_src = timed(lambda: annkin.eval_source(mech, Tt, Pt, Yt))
    nets = {}
    for tag, (l, h) in (("LF_1x8", (1, 8)), ("HF_3x32", (3, 32))):
        t0 = time.perf_counter()
        w = kcnet.train(Ttr, Ktr, l, h, epochs=20, batch=4096, lr=1e-2 if h <= 8 else 3e-3,
                        seed=1, device="cuda")
        t_train = time.perf_counter() - t0
        net = annkin.KcNet(w)
        dK = (annkin.eval_lnkc_net(net, Tv) - Kv).abs()
        om = annkin.eval_source_net(mech, net, Tt, Pt, Yt)
        rel = ((om - ex).abs()[big] / ex.abs()[big]).float()
        sel = rel[torch.randperm(rel.numel(), device=rel.device)[:1 << 20]]
        t_net = timed(lambda: annkin.eval_source_net(mech, net, Tt, Pt, Yt))
        t_lnk = timed(lambda: annkin.eval_source_lnkc(mech, Tt, Pt, Yt, Kst))
        out[tag] = {"train_s": t_train, "final_mse_standardized": w.history[-1],
                    "lnK_abs_err_median": float(dK.median()), "lnK_abs_err_max": float(dK.max()),
                    "omega_rel_err_median": float(sel.median()),
                    "omega_rel_err_p99": float(torch.quantile(sel, 0.99)),
                    "source_net_ms": t_net, "source_given_lnK_ms": t_lnk,
                    "exact_compiled_source_ms": t_src}
        nets[tag] = net
    out["accuracy_definition"] = ("FP64; omega with the network's ln K_c against the exact "
                                  "compiled source term on the 65,536 c4 states, |d|/|w| over "
                                  "entries with |w| >= 1e-6 max|w|; ln K_c errors on 2e5 "
                                  "temperatures in the training range")
    # a-posteriori (Sec. 3.1): 0-D reactors advanced with the exact ln K_c
    # and with each network; the mild variant of the same mechanism (same
    # species, thermodynamics and stoichiometry, so the networks apply)
    # allows explicit steps of 5e-16 s
    msrc = synth.make_mechanism(53, 325, ln_A_range=(8.0, 16.0), Ea_range=(20000.0, 60000.0))
    mild = annkin.Mechanism(msrc)
    m0 = 4096
    T0, P0, Y0 = (torch.tensor(a, dtype=torch.float64, device="cuda") for a in
                  synth.make_states(msrc, m0, 4242, (1000.0, 2500.0), (1.0, 20.0), 0.5))
    Te, Ye = T0.clone(), Y0.clone()
    annkin.integrate_euler(mild, Te, P0, Ye, 5e-16, 200)
    post = {"cells": m0, "dt_s": 5e-16, "steps": 200,
            "states": "T ~ U[1000, 2500] K, P ~ U[1, 20] atm, Y ~ Dirichlet(0.5)",
            "exact_max_abs_dT_K": float((Te - T0).abs().max()),
            "exact_nonfinite_cells": int((~torch.isfinite(Te)).sum())}
    for tag, net in nets.items():
        Ta, Ya = T0.clone(), Y0.clone()
        annkin.integrate_euler_net(mild, net, Ta, P0, Ya, 5e-16, 200)
        post[tag] = {"max_abs_dT_vs_exact_K": float((Ta - Te).abs().max()),
                     "median_abs_dT_vs_exact_K": float((Ta - Te).abs().median()),
                     "max_abs_dY_vs_exact": float((Ya - Ye).abs().max())}
        net.close()
    out["a_posteriori_0d"] = post
    mild.close()
    mech.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="c1_full", choices=list(synth.WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-fp64", action="store_true")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--no-deriv", action="store_true")
    ap.add_argument("--no-c2", action="store_true")
    ap.add_argument("--no-saturation", action="store_true")
    ap.add_argument("--no-pdep", action="store_true")
    ap.add_argument("--only-main", action="store_true",
                    help="time only the main FP32 leg (for profiler runs)")
    ap.add_argument("--only-deriv", action="store_true",
                    help="time only the differentiation configuration (for profiler runs)")
    ap.add_argument("--no-kc", action="store_true")
    ap.add_argument("--no-prod", action="store_true")
    ap.add_argument("--only-prod", action="store_true",
                    help="only the split-bfloat16 stoichiometric contraction")
    ap.add_argument("--only-kc", action="store_true",
                    help="time only the ln K_c network study (no training)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain 1 GiB device copy (counter calibration)")
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "this benchmark runs on one GPU: the source term shards "
                          "over cells with no exchange, so N GPUs would each run this "
                          "same single-GPU workload; run with --gpus 1"}))
        sys.exit(2)

    import torch
    if args.only_deriv:
        from paper_2008_08483_amd import annkin
        print(json.dumps({"differentiation": deriv_bench(torch, annkin)}), flush=True)
        return
    if args.only_prod:
        from paper_2008_08483_amd import annkin
        print(json.dumps({"stoich_contraction_bf16x3": prod_bench(torch, annkin)}), flush=True)
        return
    if args.only_kc:
        from paper_2008_08483_amd import annkin
        print(json.dumps({"approx_lnkc": kc_bench(torch, annkin, train=False)}), flush=True)
        return
    from paper_2008_08483_amd import annkin

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(1)
    torch.cuda.set_device(0)

    if args.copy_calibration:
        a = torch.empty(1 << 28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(5):
            b.copy_(a)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes_read": a.numel() * 4, "copy_bytes_written": b.numel() * 4}))
        return

    wl = synth.WORKLOADS[args.workload]
    src, T, P, Y = synth.workload(args.workload, dtype=np.float32)
    ns, nr, n = src.n_species, src.n_reactions, T.shape[0]
    mech = annkin.Mechanism(src)
    # mechanism load: host preprocessing and upload (synchronous), once per
    # mechanism, outside the timed steps
    load_ms = []
    for _ in range(5):
        t0 = time.perf_counter()
        extra = annkin.Mechanism(src)
        load_ms.append((time.perf_counter() - t0) * 1e3)
        extra.close()
    T32, P32, Y32 = (torch.tensor(a, device="cuda") for a in (T, P, Y))

    wall, ms, om32 = time_path(torch, annkin, mech, T32, P32, Y32, args.steps, args.warmup)
    k_avg_s = float(ms.mean()) * 1e-3
    value = n * args.steps / wall

    slots = roofline.method_slots(src.nu_f, src.nu_r)
    achieved = slots * n / k_avg_s
    traffic = measured_traffic()
    result = {
        "metric": "source-term cells/s at 53sp/325rxn (FP32 path; FP64 path, p50/p99 "
                  "latency and FP32-vs-FP64 error alongside)",
        "value": value,
        "unit": "cells/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": wall / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"{ns}sp/{nr}rxn synthetic mechanism x {n} cells, FP32 states",
                   "n_species": ns, "n_reactions": nr, "n_cells": n,
                   "mechanism_seed": synth.MECH_SEEDS[(ns, nr)], "state_seed": wl["state_seed"],
                   "layout": "T[n], P[n], Y[NS][n] (cell index fastest)"},
        "latency_ms": {"p50": float(np.percentile(ms, 50)), "p99": float(np.percentile(ms, 99)),
                       "kernel_mean": float(ms.mean())},
        "mechanism_load_ms": float(np.median(load_ms)),
        "roofline": {
            "bound": "alu",
            "achieved": achieved / 1e12,
            "peak": roofline.PEAK_VALU_SLOTS / 1e12,
            "unit": "T VALU lane-slots/s",
            "frac": achieved / roofline.PEAK_VALU_SLOTS,
            "traffic": traffic,
            "counts_per_cell": dict(zip(("transcendental", "fp32", "fp64"),
                                        roofline.method_counts(src.nu_f, src.nu_r))),
            "t_roof_us": roofline.t_valu(src.nu_f, src.nu_r, n) * 1e6,
            "frac_measured_rates": roofline.t_valu(src.nu_f, src.nu_r, n, "measured") /
                                   k_avg_s,
            "kernel": ("ak_src (compiled for the mechanism)" if mech.compiled(torch.float32)
                       else "ak::source_kernel<float>"),
            "slots_per_cell": slots,
            "hbm_GBps": roofline.hbm_bytes(ns, 4) * n / k_avg_s / 1e9,
            "hbm_frac": roofline.hbm_bytes(ns, 4) * n / k_avg_s / roofline.PEAK_HBM,
        },
    }

    if args.only_main:
        args.no_fp64 = args.no_cpu_baseline = args.no_serving = args.no_deriv = True
        args.no_c2 = args.no_saturation = args.no_pdep = args.no_kc = args.no_prod = True
    result["kernel_compiled"] = bool(mech.compiled(torch.float32))
    if not args.only_main:
        result["accuracy"] = accuracy(torch, annkin, mech, src, T, P, Y)
        # the table-driven kernel on the same launch, for comparison
        mt = annkin.Mechanism(src, kernels="table")
        result["table_kernel_fp32_ms"] = kernel_ms(torch, annkin, mt, T32, P32, Y32, reps=10)
        mt.close()
    if not args.no_fp64:
        T64, P64, Y64 = (t.double() for t in (T32, P32, Y32))
        wall64, ms64, om64 = time_path(torch, annkin, mech, T64, P64, Y64,
                                       max(5, args.steps // 2), 2)
        d = (om32.double() - om64).abs()
        ref = om64.abs()
        big = ref >= 1e-6 * ref.max()
        rel = (d[big] / ref[big]).float()
        result["fp64"] = {
            "cells_per_s": n * max(5, args.steps // 2) / wall64,
            "kernel_mean_ms": float(ms64.mean()),
            "p50_ms": float(np.percentile(ms64, 50)),
            "p99_ms": float(np.percentile(ms64, 99)),
        }
        result["err_fp32_vs_fp64"] = {
            "rel_median": float(rel.median()), "rel_p99": float(torch.quantile(
                rel[torch.randperm(rel.numel(), device=rel.device)[:1 << 20]], 0.99)),
            "definition": "|w32 - w64| / |w64| over entries with |w64| >= 1e-6 max|w64|",
        }
        del T64, P64, Y64, om64

    if args.workload == "c1_full" and not args.only_main:
        m = 65536
        wall_s, ms_s, _ = time_path(torch, annkin, mech, T32[:m].contiguous(),
                                    P32[:m].contiguous(), Y32[:, :m].contiguous(),
                                    args.steps, args.warmup)
        result["c1_65536_cells_per_s"] = m * args.steps / wall_s

    if args.workload == "c1_full" and not args.no_saturation:
        result["saturation_fp32"] = saturation(torch, annkin, mech, T32, P32, Y32)

    if args.workload == "c1_full" and not args.no_pdep:
        result["pdep_20pct"] = pdep_bench(torch, annkin, T32, P32, Y32, T, P, Y)

    if not args.no_deriv:
        result["differentiation"] = deriv_bench(torch, annkin)

    if not args.no_kc:
        result["approx_lnkc"] = kc_bench(torch, annkin)
    if not args.no_prod:
        result["stoich_contraction_bf16x3"] = prod_bench(torch, annkin)

    if not args.no_serving:
        result["serving"] = serving_bench(torch, annkin)

    if not args.no_cpu_baseline:
        result["cpu_baseline"] = cpu_baseline(src, T, P, Y)
        result["cpu_oracle_1core"] = cpu_single_core(src, T, P, Y)

    mech.close()
    del T32, P32, Y32, om32

    if args.workload == "c1_full" and not args.no_c2:
        result["c2_111x784"] = c2_bench(torch, annkin)

    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
