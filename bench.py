"""Throughput of the REWL hot path on one MI355X.

A step is one exchange interval of the whole method (Philox draws, X single-spin
attempts per walker, flatness/merge, replica exchange, interval bookkeeping) over
the workload's walkers.  Default workload: 2D Ising L=64 periodic, 16 windows with
75% overlap, 64 walkers per window (1024 walkers), exchange every 10^4 attempts,
ln f from 1 to 2^-27, Philox seed 1.

Prints one JSON line: whole-job flip attempts per second, the sweep kernel's
roofline figures (from HIP events on the library's stream), and the oracle timed on
the host cores on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

# Peaks of one MI355X (public figures): 256 CUs x 64 lanes at 2.4 GHz issue
# 3.93e13 32-bit VALU lane-operations per second (the FP64 vector rate,
# 78.6 TFLOP/s, is the same lane rate counting an FMA as two flops).
PEAK_LANE_OPS = 256 * 64 * 2.4e9
PEAK_HBM = 8.0e12

# Algorithmic lane-operations of one flip attempt inside the sweep (the draws are
# made by the RNG kernel): Ising bit-packed -- 3 row reads, 5 bit extracts, 4
# comparisons summed (12); new bin and window test (3); 2 table reads, convert,
# fused multiply-add (4); delta and the two-sided test against log u (3); the
# conditional flip, bin/histogram/base bookkeeping (5); histogram increment and
# ln g update (3).  Potts adds 2 reads and 5 comparisons for the new state.
OPS_PER_ATTEMPT = {"ising": 30, "potts": 37}

LABELS = {
    "ising8": "2D Ising L=8 periodic, 4 windows o=3/4, 1 walker/window, X=1e4, ln f to 2^-20",
    "ising32": "2D Ising L=32 periodic, 8 windows o=3/4, 16 walkers/window, X=1e4, ln f to 2^-20",
    "ising64": "2D Ising L=64 periodic, 16 windows o=3/4, 64 walkers/window, X=1e4",
    "potts32": "2D 10-state Potts L=32 periodic, 32 windows o=3/4, 128 walkers/window, X=1e4",
    "potts100": "2D 10-state Potts L=100 periodic, 77 windows of 1001 bins o=3/4, 8 walkers/window, X=1e4",
    "ising128": "2D Ising L=128 periodic, 32 windows o=3/4, 64 walkers/window, X=1e4",
    "potts64": "2D 10-state Potts L=64 periodic, 32 windows o=3/4, 128 walkers/window, X=1e4",
    "batch64": "64 independent REWL instances: Ising L 16-64 and Potts q 4/8/10 L 16-32, "
               "8-32 windows, 32-128 walkers/window, X=1e4",
}


# rocprofv3 summaries holding the HBM byte counters of a workload's sweep kernel
PROFILES = {"ising64": "k_sweep_wave_ising_L64.txt", "potts32": "k_sweep_wave_potts_q10_L32.txt",
            "batch64": "k_sweep_persist_k_rng_batch64_lane_lds53.txt",
            "ising128": "k_sweep_wave_device_ising_L128.txt",
            "potts64": "k_sweep_wave_device_potts_q10_L64.txt"}
KERNEL_SOURCES = ("paper_1407_5140_amd/csrc/rewl_kernels.hip", "paper_1407_5140_amd/csrc/rewl_device.hpp")


def profiled_traffic(wl: str, kernel: str):
    """(read, written) HBM bytes per launch from the committed counter summary, or
    None when there is none or the kernel sources changed since it was taken."""
    import hashlib
    fn = PROFILES.get(wl)
    path = os.path.join(ROOT, "profiles", fn) if fn else ""
    if not fn or not os.path.exists(path):
        return None
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    for line in open(path):
        tok = line.split()
        if len(tok) == 5 and tok[0] == "traffic" and tok[1] == kernel:
            kv = dict(t.split("=", 1) for t in tok[2:])
            if kv["source_sha256"] == h.hexdigest()[:16]:
                return int(kv["read_bytes"]), int(kv["write_bytes"])
    return None


def sweep_kernel(info: dict, tune: dict) -> str:
    """Name of the sweep kernel a handle launches (the one the roofline is taken on)."""
    if info["sweep_kind"] == "wave":
        return "k_sweep_wave"
    return "k_sweep_persist" if tune["persistent"] else "k_sweep"


def workload(name: str) -> list:
    from paper_1407_5140_amd import workloads as W
    return W.batch() if name == "batch64" else [W.single(name)]


def _sync():
    """The library's run calls return with their stream synchronised; nothing to wait for.
    (torch must not initialise its own HIP runtime in a process that uses the library.)"""


def cpu_baseline(kws: list, budget_s: float) -> dict:
    """The oracle as it stands, all host threads, a bounded number of intervals."""
    import oracle as O
    sims = [O.Sim(O.make_config(**kw)) for kw in kws]
    threads = int(os.environ.get("OMP_NUM_THREADS", "0")) or os.cpu_count() or 1
    t0 = time.perf_counter()
    for s in sims:
        s.run(1, threads=threads)
    one = time.perf_counter() - t0
    n = max(1, min(5000, int(budget_s / max(one, 1e-3))))
    t0 = time.perf_counter()
    for s in sims:
        s.run(n, threads=threads)
    dt = time.perf_counter() - t0
    att = n * sum(kw["n_windows"] * kw["m"] * kw["X"] for kw in kws)
    return {"value": att / dt, "unit": "attempts/s", "cores": threads, "kind": "oracle",
            "sample": f"{n} exchange intervals ({att:.3g} attempts) of the same workload "
                      f"after 1 warm-up interval, {dt:.1f} s"}


def exact_ln_g(kw: dict):
    """Exact ln g of the Ising workloads (stored values written by the exact routines)."""
    import numpy as np
    if kw["model"] != "ising":
        return None
    gold = os.path.join(ROOT, "tests", "golden")
    path = os.path.join(gold, f"ising_L{kw['L']}_lng.txt")
    if os.path.exists(path):
        vals = [float(l.split()[1]) for l in open(path) if l.strip() and not l.startswith("#")]
        return np.array(vals)
    path = os.path.join(gold, f"ising_q2_L{kw['L']}_counts.txt")
    if os.path.exists(path):
        import math
        cnt = [int(l.split()[1]) for l in open(path) if l.strip() and not l.startswith("#")]
        return np.array([math.log(c) if c > 0 else -math.inf for c in cnt])
    return None


def converge(rw, kw: dict, label: str, tune, max_s: float, seed: int) -> dict:
    """Wall time from the first interval until every window reached ln f <= 2^-kfinal."""
    import numpy as np
    kw = dict(kw, seed=seed)
    cfg = rw.make_config(**kw)
    g = rw.Rewl([cfg], tune=tune)
    _sync()
    t0 = time.perf_counter()
    last = t0
    done = False
    while not done and time.perf_counter() - t0 < max_s:
        done = g.run(200)
        if time.perf_counter() - last > 10:
            st = g.stats()
            print(f"[converge] {time.perf_counter() - t0:.0f} s: t={st['intervals']} min k={st['min_k']} "
                  f"windows done {st['windows_done']}/{kw['n_windows']}", file=sys.stderr, flush=True)
            last = time.perf_counter()
    dt = time.perf_counter() - t0
    st = g.stats()
    out = {"workload": label, "seed": seed, "converged": bool(done), "seconds": dt,
           "intervals": st["intervals"], "attempts": st["attempts"], "min_k": st["min_k"],
           "kfinal": kw["kfinal"], "k": [int(v) for v in st["k"]], "round_trips": int(st["round_trips_total"]),
           "ms_per_interval": dt * 1e3 / max(st["intervals"], 1)}
    if done:
        lng, join = g.concat()
        ex = exact_ln_g(kw)
        if ex is not None:
            ok = np.isfinite(ex)
            eps = np.abs(lng[ok] - ex[ok]) / np.abs(ex[ok])
            out.update(eps_max=float(eps.max()), eps_mean=float(eps.mean()),
                       abs_err_max=float(np.abs(lng[ok] - ex[ok]).max()))
    g.close()
    return out


def warm_start_study(rw, args) -> dict:
    """Time to converge with the network's warm start (ln f from 2^-k0) against
    plain flat-start REWL on the same targets: the network is trained on REWL's
    own results for smaller systems, produced in the same run."""
    from paper_1407_5140_amd import warm as Wm
    types = [("ising", 2, 16), ("ising", 2, 24), ("ising", 2, 32), ("potts", 4, 16), ("potts", 4, 24),
             ("potts", 8, 16), ("potts", 8, 24), ("potts", 10, 16), ("potts", 10, 24)]
    if args.train_types == "batch":
        types = Wm.TRAIN_TYPES            # every type of the 64-instance batch with L <= 48
    elif args.train_types == "tiny":
        types = [(mo, q, L) for (mo, q) in (("ising", 2), ("potts", 4), ("potts", 8), ("potts", 10))
                 for L in (8, 12)]
    log = lambda m: print(f"[warm] {m}", file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    kws = Wm.training_workload(types, m=32 if args.train_types != "tiny" else 16, kfinal=args.train_kfinal)
    g, res = Wm.run_to_convergence(kws, args.max_seconds, log=log)
    ok = [r["converged"] for r in res]
    x, t = Wm.training_rows(g, kws, ok)
    g.close()
    t_train = time.perf_counter() - t0
    log(f"training set: {sum(ok)}/{len(kws)} instances converged to 2^-{args.train_kfinal}, "
        f"{len(t)} rows, {t_train:.1f} s")
    net, info = Wm.train(x, t, steps=args.mlp_steps, batch=4096, lr=1e-3)
    log(f"network: {info}")
    known = {"potts16": dict(model="potts", q=10, L=16, n_windows=8, m=16),
             "ising24": dict(model="ising", q=2, L=24, n_windows=8, m=16),
             "potts32": dict(model="potts", q=10, L=32, n_windows=16, m=32),
             "ising48": dict(model="ising", q=2, L=48, n_windows=32, m=32),
             "ising64": dict(model="ising", q=2, L=64, n_windows=16, m=64),
             # the paper's Potts lattice with windows narrowed towards the ground state
             "potts100t": dict(model="potts", q=10, L=100, n_windows=90, m=8)}
    targets = [dict(known[t], kfinal=args.kfinal, X=10000, seed=sd) for t in args.warm_targets.split(",")
               for sd in range(1, args.warm_seeds + 1)]
    for kw in targets:
        if kw["L"] == 100:
            kw["windows"] = tilted_windows(rw, kw)
    modes = args.warm_modes.split(",")
    out = []
    for kw in targets:
        label = f"{kw['model']} q={kw['q']} L={kw['L']} h={kw['n_windows']} m={kw['m']} seed={kw['seed']}"
        tab = Wm.warm_table(net, kw)
        k0 = args.k0 if args.k0 >= 0 else Wm.suggest_k0(info["rms"], kw["L"] ** 2)
        row = {"workload": label, "kfinal": kw["kfinal"], "k0_warm": k0}
        ex = exact_ln_g(kw)
        for mode in modes:
            k = dict(kw, k0=k0 if mode == "warm" else 0)
            gg, rr = Wm.run_to_convergence([k], args.target_seconds,
                                           warm_tables=[tab] if mode == "warm" else None, log=log)
            r = dict(rr[0])
            if ex is not None and r["converged"]:
                lng, _ = gg.concat(0)
                okb = np.isfinite(ex)
                eps = np.abs(lng[okb] - ex[okb]) / np.abs(ex[okb])
                r["eps_max"] = float(eps.max())
                r["eps_mean"] = float(eps.mean())
            gg.close()
            row[mode] = r
            log(f"{label} {mode}: {r}")
        if "warm" in row and "plain" in row and row["warm"]["converged"] and row["plain"]["converged"]:
            row["speedup"] = row["plain"]["seconds"] / row["warm"]["seconds"]
        out.append(row)
    net.close()
    return {"mode": "warm-start vs plain REWL", "train": {"instances": len(kws), "kfinal": args.train_kfinal,
            "converged": int(sum(ok)), "rows": int(len(t)), "seconds": t_train},
            "network": info, "targets": out}


def warm_error_study(rw, args) -> dict:
    """How accurate a starting table must be for a given initial ln f = 2^-k0:
    a converged run (ln f -> 2^-20) of 10-state Potts L=16 serves as the true
    table; warm tables are that table plus a smooth error of amplitude delta
    (three periods of a sine over the energy range, rounded to 2^-16), and each
    (delta, k0) pair runs to 2^-kfinal on the same seed.  Counted in intervals."""
    from paper_1407_5140_amd import warm as Wm
    log = lambda m: print(f"[warm-error] {m}", file=sys.stderr, flush=True)
    kw = dict(model="potts", q=10, L=16, n_windows=4, m=8, X=2000, seed=3)
    g, res = Wm.run_to_convergence([dict(kw, kfinal=20)], args.max_seconds, poll=10)
    truth, _ = g.concat(0)
    g.close()
    W = truth.size
    b = np.arange(W)
    base = np.where(np.isfinite(truth), truth, 0.0)
    out = {"mode": "warm-table error against initial ln f", "workload": "2D 10-state Potts L=16, h=4, m=8, "
           f"X=2000, ln f -> 2^-{args.kfinal}", "reference_intervals": res[0]["intervals"], "runs": []}
    plain = None
    for delta in [float(v) for v in args.error_deltas.split(",")]:
        tab = base + delta * np.sin(6 * np.pi * b / (W - 1))
        tab = np.round(tab * 65536.0) / 65536.0
        for k0 in [int(v) for v in args.error_k0s.split(",")]:
            k = dict(kw, kfinal=args.kfinal, k0=k0)
            gg, rr = Wm.run_to_convergence([k], args.target_seconds, warm_tables=[tab], poll=10)
            gg.close()
            r = {"delta": delta, "k0": k0, "converged": rr[0]["converged"], "intervals": rr[0]["intervals"],
                 "seconds": rr[0]["seconds"]}
            out["runs"].append(r)
            log(str(r))
    gg, rr = Wm.run_to_convergence([dict(kw, kfinal=args.kfinal)], args.target_seconds, poll=10)
    gg.close()
    out["plain"] = {"intervals": rr[0]["intervals"], "seconds": rr[0]["seconds"], "converged": rr[0]["converged"]}
    log(f"plain: {out['plain']}")
    return out


def exchange_study(rw, args) -> dict:
    """Replica exchange on against off, and the exchange interval, on the paper's
    kind of test (Sec. IV: a Potts model split into 15 windows): attempts per
    walker until every window reaches ln f = 2^-kfinal, over several seeds.  All
    settings run as independent instances of one batch; the count of attempts is
    exact and machine-independent."""
    from paper_1407_5140_amd import warm as Wm
    base = dict(model="potts", q=10, L=args.study_L, n_windows=15, m=1, kfinal=args.study_kfinal)
    settings = [("exchange", 1000), ("exchange", 10000), ("exchange", 100000), ("none", 10000)]
    kws, tags = [], []
    for mode, X in settings:
        for sd in range(1, args.study_seeds + 1):
            kws.append(dict(base, X=X, seed=100 + sd, exchange=(mode == "exchange")))
            tags.append((mode, X))
    log = lambda m: print(f"[exchange] {m}", file=sys.stderr, flush=True)
    g, res = Wm.run_to_convergence(kws, args.max_seconds, tune=rw.make_tune(use_graph=1, poll_every=50),
                                   log=log)
    trips = [int(g.stats(i)["round_trips_total"]) for i in range(len(kws))]
    g.close()
    rows = []
    for mode, X in settings:
        sel = [i for i, t in enumerate(tags) if t == (mode, X)]
        att = [res[i]["intervals"] * X for i in sel if res[i]["converged"]]
        rows.append({"exchange": mode == "exchange", "X": X, "converged": sum(res[i]["converged"] for i in sel),
                     "attempts_per_walker": att,
                     "min_k_unconverged": [res[i]["min_k"] for i in sel if not res[i]["converged"]],
                     "attempts_unconverged": [res[i]["intervals"] * X for i in sel if not res[i]["converged"]],
                     "round_trips": [trips[i] for i in sel],
                     "median": float(np.median(att)) if len(att) == len(sel) else None})
    ref = next(r for r in rows if not r["exchange"])["median"]
    for r in rows:
        r["speedup_vs_no_exchange"] = (ref / r["median"]) if (ref and r["median"]) else None
    return {"mode": "replica exchange on/off", "workload": f"Potts q=10 L={args.study_L}, 15 windows o=3/4, "
            f"1 walker/window, ln f 1 -> 2^-{args.study_kfinal}", "settings": rows}


def mlp_bench(rw, args) -> dict:
    """Training throughput of the DOS network (3 x 256 GELU, batch 4096) on rows
    shaped like the warm-start data; matrix-core work per step: six 4096 x 256 x 256
    products (two forward, two weight gradients, two input gradients)."""
    rng = np.random.default_rng(1)
    n = 16384
    L = rng.choice([16.0, 24.0, 32.0, 48.0], n)
    x = np.stack([rng.uniform(-2, 2, n), 1.0 / L, rng.choice([2.0, 4.0, 8.0, 10.0], n)], axis=1)
    t = np.log(2.0) * (1 - (x[:, 0] / 2) ** 2) + 0.01 * x[:, 1]
    net = rw.Mlp(3, 256, 3, max_batch=4096, seed=1)
    net.fit(x, t, args.mlp_warmup_steps, batch=4096, lr=1e-3)
    t0 = time.perf_counter()
    loss = net.fit(x, t, args.mlp_steps, batch=4096, lr=1e-3)
    dt = time.perf_counter() - t0
    net.close()
    flops = 6 * 2 * 4096 * 256 * 256
    return {"mode": "DOS network training", "batch": 4096, "steps": args.mlp_steps,
            "ms_per_step": dt * 1e3 / args.mlp_steps, "matrix_tflops_per_s": flops * args.mlp_steps / dt / 1e12,
            "gemm_flops_per_step": flops, "last_loss": loss}


def balanced_study(rw, args) -> dict:
    """Windows of equal width against windows balanced by a pilot run (Sec. V:
    windows that converge at a similar pace).  The pilot runs the equal layout
    until every window has halved ln f k_pilot times; a window's difficulty is
    sqrt(intervals per halving over the pilot's second half) spread over its bins,
    and rewl_balanced_layout gives windows of equal total difficulty.  Then both
    layouts run to ln f = 2^-kfinal on the same seed."""
    from paper_1407_5140_amd import warm as Wm
    kw = dict(model="ising", q=2, L=args.study_L_balanced, n_windows=8, m=16, kfinal=args.kfinal_balanced,
              X=10000, seed=1)
    log = lambda m: print(f"[balanced] {m}", file=sys.stderr, flush=True)
    cfg = rw.make_config(**kw)
    W, WB, lo, hi = rw.rewl_layout(cfg)
    h, kp = kw["n_windows"], args.k_pilot
    g = rw.Rewl([rw.make_config(**dict(kw, kfinal=kp))], tune=rw.make_tune(poll_every=20))
    reached = np.full((h, kp + 1), -1, np.int64)
    t0 = time.perf_counter()
    while True:
        done = g.run(20)
        st = g.state()
        for a in range(h):
            for kk in range(int(st["k"][a]) + 1):
                if reached[a, kk] < 0:
                    reached[a, kk] = st["t"]
        if done or time.perf_counter() - t0 > args.max_seconds:
            break
    g.close()
    t_pilot = time.perf_counter() - t0
    half = kp // 2
    per = (reached[:, kp] - reached[:, half]) / (kp - half)
    rho_w = np.sqrt(np.maximum(per, 1.0)) / (hi - lo + 1)
    rho = np.zeros(W)
    cnt = np.zeros(W)
    for a in range(h):
        rho[lo[a]:hi[a] + 1] += rho_w[a]
        cnt[lo[a]:hi[a] + 1] += 1
    rho /= cnt
    blo, bhi = rw.rewl_balanced_layout(cfg, rho)
    log(f"pilot {t_pilot:.1f} s, intervals per halving by window {per.tolist()}; balanced windows "
        f"{list(zip(blo.tolist(), bhi.tolist()))}")
    ex = exact_ln_g(kw)
    out = {"mode": "equal against balanced windows", "workload": f"Ising L={kw['L']} h=8 m=16, ln f -> "
           f"2^-{kw['kfinal']}", "pilot": {"k_pilot": kp, "seconds": t_pilot,
           "intervals_per_halving": per.tolist()}, "balanced_windows": [blo.tolist(), bhi.tolist()]}
    for name, wins in (("equal", None), ("balanced", (blo, bhi))):
        gg, res = Wm.run_to_convergence([dict(kw, windows=wins) if wins is not None else kw],
                                        args.target_seconds, log=log)
        r = dict(res[0])
        if r["converged"] and ex is not None:
            lng, _ = gg.concat(0)
            okb = np.isfinite(ex)
            eps = np.abs(lng[okb] - ex[okb]) / np.abs(ex[okb])
            r.update(eps_max=float(eps.max()), eps_mean=float(eps.mean()))
        gg.close()
        out[name] = r
        log(f"{name}: {r}")
    if out["equal"]["converged"] and out["balanced"]["converged"]:
        out["speedup"] = out["equal"]["seconds"] / out["balanced"]["seconds"]
    return out


def ensemble_study(rw, args) -> dict:
    """The paper's 10-state Potts L=100 workload (77 windows of 1001 bins, overlap
    3/4, m walkers per window) as n independent runs in one batch, run to
    ln f = 2^-kfinal or the time limit; then the error analysis of Sec. II.B
    (mean of the n pieces per window + R bootstrap resamples, rewl_ensemble) and
    the specific heat of every row (rewl_thermo) near the transition."""
    from paper_1407_5140_amd import workloads as Wl
    log = lambda m: print(f"[ensemble] {m}", file=sys.stderr, flush=True)
    n = args.ens_runs
    base = dict(Wl.single("potts100"), kfinal=args.ens_kfinal)
    if args.m:
        base["m"] = args.m
    if args.ens_h:
        base["n_windows"] = args.ens_h
    if args.ens_windows == "ground-tilt":
        base["windows"] = tilted_windows(rw, base)
        log(f"windows {len(base['windows'][0])}, widths "
            f"{(base['windows'][1] - base['windows'][0] + 1).tolist()}")
    kws = [dict(base, seed=1 + j) for j in range(n)]
    t0 = time.perf_counter()
    g = rw.Rewl([rw.make_config(**kw) for kw in kws], tune=rw.make_tune(poll_every=50))
    t_create = time.perf_counter() - t0
    info = g.info()
    log(f"{n} runs x {base['n_windows']} windows x {base['m']} walkers, {info['sweep_kind']} sweep, "
        f"create {t_create:.1f} s")
    t0 = time.perf_counter()
    last = t0
    done = False
    while not done and time.perf_counter() - t0 < args.max_seconds:
        done = g.run(50)
        if time.perf_counter() - last > 30:
            last = time.perf_counter()
            sts = [g.stats(i) for i in range(n)]
            log(f"{last - t0:.0f} s: intervals {sts[0]['intervals']}, min k "
                f"{[s['min_k'] for s in sts]}, windows done {[s['windows_done'] for s in sts]}")
    t_run = time.perf_counter() - t0
    sts = [g.stats(i) for i in range(n)]
    attempts = sum(s["attempts"] for s in sts)
    log(f"run {t_run:.1f} s, {attempts / t_run:.4g} attempts/s, converged {done}")
    # windows that have not reached the final ln f, with their energy ranges per spin
    _, _, wlo, whi = g.layouts[0]
    N = base["L"] ** 2
    behind = []
    for i in range(n):
        k = g.state(i)["k"]
        behind.append([[int(a), int(k[a]), round((wlo[a] - 2 * N) / N, 4), round((whi[a] - 2 * N) / N, 4)]
                       for a in range(len(k)) if k[a] < base["kfinal"]])
    log(f"windows behind (window, k, E/N from, to): {behind}")
    R = args.ens_R
    t0 = time.perf_counter()
    rows, joins = g.ensemble(list(range(n)), R=R, seed=1)
    t_ens = time.perf_counter() - t0
    g.close()
    T = np.linspace(args.ens_tmin, args.ens_tmax, args.ens_nT)
    t0 = time.perf_counter()
    u, c, f = rw.rewl_thermo("potts", base["L"], rows, T)
    t_th = time.perf_counter() - t0
    peak = T[np.argmax(c, axis=1)]
    cmax = c.max(axis=1)
    out = {"mode": "n-run ensemble, bootstrap and specific heat",
           "workload": f"2D 10-state Potts L={base['L']}, {base['n_windows']} windows o=3/4, "
                       f"m={base['m']}, ln f -> 2^-{base['kfinal']}, {n} runs",
           "converged": bool(done), "run_seconds": t_run, "attempts_per_s": attempts / t_run,
           "min_k": [s["min_k"] for s in sts], "intervals": sts[0]["intervals"],
           "windows_behind": behind,
           "resamples": R, "ensemble_seconds": t_ens, "thermo_seconds": t_th,
           "thermo_grid": [float(T[0]), float(T[-1]), int(T.size)],
           "T_peak": float(peak[0]), "T_peak_err": float(np.std(peak[1:])) if R > 1 else None,
           "c_max": float(cmax[0]), "c_max_err": float(np.std(cmax[1:])) if R > 1 else None,
           "joins_spread": float(np.mean(np.std(joins[1:], axis=0))) if R > 1 else None}
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = ensemble_cpu_baseline(kws, n, R, T, args.cpu_budget)
    log(json.dumps(out))
    return out


def tilted_windows(rw, kw):
    """Windows narrowed towards the slow ground levels: the library's difficulty
    model near the ground levels (rewl_tilt_density) through rewl_balanced_layout."""
    return rw.tilted_layout(rw.make_config(**kw))


def ensemble_cpu_baseline(kws, n, R, T, budget_s) -> dict:
    """The oracle on the host beside the device: its REWL run on one of the n runs
    (bounded intervals), and its mean + bootstrap and canonical averages on
    synthetic tables of the same shape, timed on a few rows and scaled to R + 1."""
    import oracle as O
    from oracle import ensemble as EN
    res = {"sweep": cpu_baseline([kws[0]], budget_s)}
    c = O.make_config(**kws[0])
    W = O.n_bins(c)
    lo, hi = O.layout(c)
    WB = int((hi - lo).max()) + 1
    rng = np.random.default_rng(0)
    b = np.arange(W)
    tab = 3000.0 * np.sin(np.pi * b / (W - 1))
    runs = np.zeros((n, len(lo), WB))
    for j in range(n):
        t = tab + rng.normal(0, 0.02, W) + 17.0 * j
        for a in range(len(lo)):
            runs[j, a, : hi[a] - lo[a] + 1] = t[lo[a]: hi[a] + 1]
    mask = O.mask_rule(c)
    r_s = 8
    t0 = time.perf_counter()
    rows, _ = EN.ensemble(c, mask, runs, R=r_s - 1, seed=1)
    t_ens = (time.perf_counter() - t0) * (R + 1) / r_s
    t0 = time.perf_counter()
    EN.canonical("potts", kws[0]["L"], rows[0], T)
    t_th = (time.perf_counter() - t0) * (R + 1)
    res["ensemble_seconds"] = t_ens
    res["thermo_seconds"] = t_th
    res["sample"] = (f"ensemble: {r_s} rows timed, scaled to {R + 1}; canonical averages: one row of "
                     f"{T.size} temperatures timed, scaled to {R + 1} rows; one thread (numpy/C)")
    return res


def headline_study(rw, args) -> dict:
    """The warm-start comparison to ln f = 2^-27 (~1e-8) with the DOS error gate.

    The network is trained on REWL's own results (ln f -> 2^-16) for Ising and
    10-state Potts lattices smaller than the target, produced in this run.  The
    target (Ising, exact DOS known) runs n seeds plain (ln f from 1) and n seeds
    warm (the network's table, ln f from 2^-k0), each group in its own handle so
    that each has the GPU to itself; time to converge = wall time until every
    window of every seed of the group reached 2^-kfinal.  Accuracy: eps = |ln g^ -
    ln g| / ln g over the levels that occur (max and mean), per run and for the
    n-run mean of the pieces joined by the paper's rule (Sec. II.B), the gate
    being max eps <= 5e-3."""
    from paper_1407_5140_amd import warm as Wm
    log = lambda m: print(f"[headline] {m}", file=sys.stderr, flush=True)
    L, h, m, kf, n = args.hl_L, args.hl_h, args.hl_m, args.hl_kfinal, args.hl_seeds
    flat = tuple(int(v) for v in args.hl_flat.split(","))
    types = [(mo, q, Lt) for (mo, q) in (("ising", 2), ("potts", 10)) for Lt in (8, 12, 16, 20) if Lt < L]
    t0 = time.perf_counter()
    kws = [dict(model=mo, q=q, L=Lt, n_windows=4, m=32, kfinal=16, X=10000, seed=3000 + i)
           for i, (mo, q, Lt) in enumerate(types)]
    g, res = Wm.run_to_convergence(kws, args.max_seconds, log=log)
    okr = [r["converged"] for r in res]
    x, t = Wm.training_rows(g, kws, okr)
    g.close()
    t_data = time.perf_counter() - t0
    net, info = Wm.train(x, t, steps=args.mlp_steps, batch=4096, lr=1e-3)
    log(f"training: {sum(okr)}/{len(kws)} instances, {len(t)} rows, {t_data:.1f} s; network {info}")
    target = dict(model="ising", q=2, L=L, n_windows=h, m=m, kfinal=kf, X=10000, flat=flat)
    tab = Wm.warm_table(net, target)
    k0 = args.k0 if args.k0 >= 0 else Wm.suggest_k0(info["rms"], L * L)
    net.close()
    ex = exact_ln_g(target)
    ok = np.isfinite(ex)

    def eps(lng):
        e = np.abs(lng[ok] - ex[ok]) / np.abs(ex[ok])
        return {"eps_max": float(e.max()), "eps_mean": float(e.mean()),
                "abs_err_max": float(np.abs(lng[ok] - ex[ok]).max())}

    groups = {}
    for mode in ("plain", "warm"):
        tk = [dict(target, seed=sd, k0=k0 if mode == "warm" else 0) for sd in range(1, n + 1)]
        ts = time.perf_counter()
        gg, rr = Wm.run_to_convergence(tk, args.max_seconds, warm_tables=[tab] * n if mode == "warm" else None,
                                       poll=100, log=log)
        wall = time.perf_counter() - ts
        conv = all(r["converged"] for r in rr)
        runs = []
        for i, r in enumerate(rr):
            row = dict(seed=i + 1, converged=r["converged"], intervals=r["intervals"], seconds=r["seconds"],
                       min_k=r["min_k"])
            if r["converged"]:
                row.update(eps(gg.concat(i)[0]))
            runs.append(row)
        grp = dict(k0=k0 if mode == "warm" else 0, converged=conv, seconds=wall if conv else None,
                   seconds_limit=None if conv else wall, runs=runs)
        if conv:
            mean_rows, _ = gg.ensemble(list(range(n)), R=0)
            grp["n_run_mean"] = eps(mean_rows[0])
            grp["gate_met"] = grp["n_run_mean"]["eps_max"] <= 5e-3
        gg.close()
        groups[mode] = grp
        log(f"{mode}: converged {conv}, {wall:.0f} s, n-run mean {grp.get('n_run_mean')}")
    out = {"mode": "headline: warm start vs plain REWL to 2^-%d" % kf,
           "workload": f"Ising L={L} periodic, h={h}, m={m}, o=3/4, flatness {flat[0]}/{flat[1]}, X=1e4, "
                       f"{n} seeds per group, ln f 1 (plain) or 2^-{k0} (warm) -> 2^-{kf}",
           "train": {"types": types, "instances": len(kws), "converged": int(sum(okr)), "rows": int(len(t)),
                     "seconds": t_data}, "network": info, "groups": groups}
    if groups["plain"]["converged"] and groups["warm"]["converged"]:
        out["speedup_warm_over_plain"] = groups["plain"]["seconds"] / groups["warm"]["seconds"]
        out["speedup_with_training"] = groups["plain"]["seconds"] / (groups["warm"]["seconds"] + t_data
                                                                      + info["seconds"])
    return out


def target_study(rw, args) -> dict:
    """Warm start against plain REWL on a large target.

    The network is trained on REWL's own results (ln f -> 2^-16) for every type of
    the 64-instance batch with L <= 48, produced in this run (skipped when every
    instance is plain).  The target then runs once per entry of --ts-k0: 0 is plain
    (ln f from 1), k0 > 0 the network's table with ln f from 2^-k0, -1 the k0 the
    table's error suggests.  All of them are instances of one handle, so every sweep
    launch covers all of them and they share one clock (a single entry has the GPU
    to itself).  Reported: per-window k of every instance at regular times, the
    first time each instance had every window at k >= K, and for converged Ising
    instances the error against the exact DOS."""
    from paper_1407_5140_amd import warm as Wm
    log = lambda m: print(f"[target] {m}", file=sys.stderr, flush=True)
    target = dict(workload(args.ts_target)[0], seed=args.ts_seed)
    if args.windows == "tilted":
        target["windows"] = tilted_windows(rw, target)
    asked = [int(v) for v in args.ts_k0.split(",")]
    out = {"mode": "warm start vs plain on a large target, one handle"}
    tab, info = None, None
    if any(v != 0 for v in asked):
        t0 = time.perf_counter()
        kws = Wm.training_workload(Wm.TRAIN_TYPES, m=32, kfinal=16)
        g, res = Wm.run_to_convergence(kws, args.max_seconds, log=log)
        okr = [r["converged"] for r in res]
        x, t = Wm.training_rows(g, kws, okr)
        g.close()
        t_data = time.perf_counter() - t0
        net, info = Wm.train(x, t, steps=args.mlp_steps, batch=4096, lr=1e-3)
        log(f"training: {sum(okr)}/{len(kws)} instances, {len(t)} rows, {t_data:.1f} s; network {info}")
        tab = Wm.warm_table(net, target)
        net.close()
        out["train"] = {"types": Wm.TRAIN_TYPES, "converged": int(sum(okr)), "rows": int(len(t)),
                        "seconds": t_data}
        out["network"] = info
    k0s = [v if v >= 0 else Wm.suggest_k0(info["rms"], target["L"] ** 2) for v in asked]
    cfgs = [rw.make_config(**dict(target, k0=k0)) for k0 in k0s]
    gg = rw.Rewl(cfgs, tune=rw.make_tune(autotune=1, use_graph=1, poll_every=1 << 20))
    for i, k0 in enumerate(k0s):
        if k0 > 0:
            gg.set_initial_lng(tab, i)
    log(f"{args.ts_target}: instances with k0 {k0s}, tune {gg.tune()}, info {gg.info()}")
    h = target["n_windows"]
    reached = [dict() for _ in k0s]          # K -> (seconds, intervals) of the first all-windows >= K
    samples, last = [], -1e9
    ts = time.perf_counter()
    while True:
        all_done = gg.run(200)
        now = time.perf_counter() - ts
        sts = [gg.stats(i) for i in range(len(k0s))]
        for i, st in enumerate(sts):
            for K in range(0, int(min(st["k"])) + 1):
                reached[i].setdefault(K, (now, st["intervals"]))
        if now - last >= args.ts_sample or all_done or now > args.ts_seconds:
            samples.append({"seconds": now, "intervals": sts[0]["intervals"],
                            "k": [[int(v) for v in st["k"]] for st in sts],
                            "round_trips": [int(st["round_trips_total"]) for st in sts]})
            log(f"{now:.0f} s, {sts[0]['intervals']} intervals: min k {[int(min(st['k'])) for st in sts]}, "
                f"mean k {[round(float(np.mean(st['k'])), 2) for st in sts]}, windows done "
                f"{[int(st['windows_done']) for st in sts]}/{h}")
            last = now
        if all_done or now > args.ts_seconds:
            break
    names = ["plain" if k0 == 0 else f"warm k0={k0}" for k0 in k0s]
    kf = target["kfinal"]
    ex = exact_ln_g(target)
    runs = []
    for i in range(len(k0s)):
        r = {"instance": names[i], "converged": kf in reached[i],
             "seconds": reached[i][kf][0] if kf in reached[i] else None,
             "intervals": reached[i][kf][1] if kf in reached[i] else None}
        if ex is not None and r["converged"]:
            lng, _ = gg.concat(i)
            ok = np.isfinite(ex)
            e = np.abs(lng[ok] - ex[ok]) / np.abs(ex[ok])
            big = ex[ok] > 10
            r.update(eps_max=float(e.max()), eps_mean=float(e.mean()),
                     abs_err_max_lng_above_10=float(np.abs(lng[ok] - ex[ok])[big].max()))
        runs.append(r)
        log(f"{names[i]}: {r}")
    gg.close()
    levels = sorted(set().union(*[r.keys() for r in reached]))
    first = {str(K): [reached[i].get(K, (None, None))[0] for i in range(len(k0s))] for K in levels}
    out.update({"workload": f"{LABELS.get(args.ts_target, args.ts_target)}; windows {args.windows}; "
                            f"ln f 1 (plain) or 2^-k0 (warm) -> 2^-{kf}; seed {args.ts_seed}",
                "instances": names, "k0": k0s, "seconds_limit": args.ts_seconds, "runs": runs,
                "first_all_windows_at_k": first, "samples": samples})
    return out


def accuracy_study(rw, args) -> dict:
    """Where the DOS error of Ising runs comes from (Sec. II.B joins against the pieces
    themselves), judged against the exact DOS.  n seeds of one workload run in one
    handle to ln f = 2^-kfinal.  Per run: the normalised error eps = |ln g^ - ln g| / ln g
    (mean, max); per piece, its error r(E) = piece - exact over the levels that occur,
    split into a constant (free: the joins remove it) and the rest; the change of r
    between the piece's two join points (the joined DOS accumulates these changes from
    the middle of the range to its ends); and the error of the same pieces joined by
    the paper's rule after averaging the n runs' pieces window by window (Sec. II.B's
    n-run mean), as rewl_ensemble does."""
    L, h, m = args.acc_L, args.acc_h, args.acc_m
    kw0 = dict(model="ising", q=2, L=L, n_windows=h, m=m, kfinal=args.acc_kfinal, X=10000)
    if args.flat and args.flat_rule == "mean":
        kw0["flat"] = tuple(int(v) for v in args.flat.split(","))
    elif args.flat:
        kw0.update(flat_rule=args.flat_rule, flat=tuple(int(v) for v in args.flat.split(",")))
    if args.windows == "tilted":
        kw0["windows"] = tilted_windows(rw, dict(kw0, seed=1))
    seeds = list(range(1, args.acc_seeds + 1))
    kws = [dict(kw0, seed=sd) for sd in seeds]
    ex = exact_ln_g(kw0)
    ok = np.isfinite(ex)
    g = rw.Rewl([rw.make_config(**kw) for kw in kws], tune=rw.make_tune(poll_every=200))
    t0 = time.perf_counter()
    last = t0
    done = False
    while not done and time.perf_counter() - t0 < args.max_seconds:
        done = g.run(200)
        if time.perf_counter() - last > 20:
            sts = [g.stats(i) for i in range(len(kws))]
            print(f"[accuracy] {time.perf_counter() - t0:.0f} s: min k {[s['min_k'] for s in sts]}",
                  file=sys.stderr, flush=True)
            last = time.perf_counter()
    secs = time.perf_counter() - t0
    W, WB, lo, hi = rw.rewl_layout(rw.make_config(**kws[0]))

    def eps(lng):
        e = np.abs(lng[ok] - ex[ok]) / np.abs(ex[ok])
        return float(e.mean()), float(e.max()), float(np.abs(lng[ok] - ex[ok]).max())

    runs = []
    for i in range(len(kws)):
        st = g.stats(i)
        pieces = g.pieces(i)
        lng, join = g.concat(i)
        pc = []
        for a in range(h):
            b = np.arange(lo[a], hi[a] + 1)
            occ = ok[b]
            r = pieces[a][: hi[a] - lo[a] + 1][occ] - ex[b][occ]
            c = r.mean()
            rr = np.full(b.size, np.nan)
            rr[occ] = r - c
            ends = [join[a - 1] if a > 0 else lo[a], join[a] if a < h - 1 else hi[a]]
            drift = float(rr[ends[1] - lo[a]] - rr[ends[0] - lo[a]]) if np.all(np.isfinite(rr[[e - lo[a] for e in ends]])) else None
            pc.append(dict(rms=float(np.sqrt(np.mean((r - c) ** 2))), max=float(np.abs(r - c).max()),
                           drift_between_joins=drift))
        e_mean, e_max, d_max = eps(lng)
        d = lng - ex
        runs.append(dict(seed=seeds[i], intervals=st["intervals"], min_k=st["min_k"], eps_mean=e_mean,
                         eps_max=e_max, abs_err_max=d_max, err_E0=float(d[0]), err_Emax=float(d[W - 1]),
                         err_low_end=[round(float(v), 4) for v in d[:24][ok[:24]]],
                         err_high_end=[round(float(v), 4) for v in d[W - 24:][ok[W - 24:]]],
                         joins=[int(j) for j in join], pieces=pc, round_trips=int(st["round_trips_total"])))
    out = dict(mode="accuracy", workload=f"Ising L={L}, h={h}, m={m}, ln f -> 2^-{args.acc_kfinal}"
               + (f", windows {args.windows}" if args.windows != "equal" else "")
               + (f", flatness {kw0.get('flat_rule', 'mean')} {kw0.get('flat')}" if args.flat else ""),
               seeds=seeds, converged=bool(done), seconds=secs, runs=runs)
    if done:
        mean_rows, _ = g.ensemble(list(range(len(kws))), R=0)
        out["n_run_mean"] = dict(zip(("eps_mean", "eps_max", "abs_err_max"), eps(mean_rows[0])))
        d = mean_rows[0] - ex
        out["n_run_mean"].update(err_E0=float(d[0]), err_Emax=float(d[W - 1]),
                                 err_low_end=[round(float(v), 4) for v in d[:24][ok[:24]]],
                                 err_high_end=[round(float(v), 4) for v in d[W - 24:][ok[W - 24:]]])
    g.close()
    return out


def main(argv=None):
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="ising64", choices=sorted(LABELS))
    ap.add_argument("--autotune", action="store_true")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="default run only: skip the batch throughput and the Ising L=8 time-to-converge keys")
    ap.add_argument("--sweep", default="auto", choices=["auto", "lane", "wave"])
    ap.add_argument("--converge", action="store_true",
                    help="run to convergence and print time-to-converge and DOS error")
    ap.add_argument("--max-seconds", type=float, default=600.0)
    ap.add_argument("--seeds", default="1")
    ap.add_argument("--calib-copy-mib", type=int, default=0,
                    help="only copy a device buffer of this size and exit (a kernel of known "
                         "traffic for scaling the HBM byte counters)")
    ap.add_argument("--wpb", type=int, default=0, help="walkers per block (0 = library choice)")
    ap.add_argument("--persistent", action="store_true", help="lane sweep: persistent grid over a tile queue")
    ap.add_argument("--map-log2", type=int, default=0,
                    help="wave sweep: at most 2^v site-map entries per walker (6..12; 0 = library's choice)")
    ap.add_argument("--placement", default="auto", choices=["auto", "lds", "device"],
                    help="wave sweep: where the walkers' counts live while it runs")
    ap.add_argument("--lds-kb", type=int, default=0,
                    help="lane sweep: cap on a tile's LDS in KiB (0 = the device limit)")
    ap.add_argument("--flat-rule", default="mean", choices=["mean", "visits"],
                    help="--converge: flatness rule (mean: min H >= num/den of the mean; "
                         "visits: H >= (num/den)/sqrt(ln f) for every level, Eq. (8))")
    ap.add_argument("--flat", default="", help="--converge: flatness parameter num,den")
    ap.add_argument("--m", type=int, default=0, help="--converge: walkers per window override")
    ap.add_argument("--kfinal-override", type=int, default=0, help="--converge: final ln f exponent")
    ap.add_argument("--windows", default="equal", choices=["equal", "tilted"],
                    help="--converge: tilted = narrowed towards the slow ends (Ising both, Potts the ground level)")
    ap.add_argument("--mlp-bench", action="store_true", help="time the DOS network's training steps")
    ap.add_argument("--mlp-warmup-steps", type=int, default=20)
    ap.add_argument("--balanced-study", action="store_true",
                    help="time to converge with equal windows against pilot-balanced windows")
    ap.add_argument("--study-L-balanced", type=int, default=32)
    ap.add_argument("--kfinal-balanced", type=int, default=20)
    ap.add_argument("--k-pilot", type=int, default=12)
    ap.add_argument("--warm-error-study", action="store_true",
                    help="intervals to converge from tables of known error against the initial ln f")
    ap.add_argument("--error-deltas", default="0.1,1,10")
    ap.add_argument("--error-k0s", default="0,6,10")
    ap.add_argument("--exchange-study", action="store_true",
                    help="attempts to converge with replica exchange on/off and several intervals")
    ap.add_argument("--study-L", type=int, default=24)
    ap.add_argument("--study-kfinal", type=int, default=14)
    ap.add_argument("--study-seeds", type=int, default=4)
    ap.add_argument("--headline", action="store_true",
                    help="warm start vs plain to 2^-kfinal on an Ising target with the DOS error gate")
    ap.add_argument("--hl-L", type=int, default=24)
    ap.add_argument("--hl-h", type=int, default=8)
    ap.add_argument("--hl-m", type=int, default=64)
    ap.add_argument("--hl-kfinal", type=int, default=27)
    ap.add_argument("--hl-seeds", type=int, default=8)
    ap.add_argument("--hl-flat", default="19,20")
    ap.add_argument("--target-study", action="store_true",
                    help="warm start against plain on a large target at equal GPU time")
    ap.add_argument("--ts-target", default="potts64")
    ap.add_argument("--ts-k0", default="0,-1,10",
                    help="one instance per value: 0 plain, k0 > 0 warm from 2^-k0, -1 k0 from the network's error")
    ap.add_argument("--ts-seconds", type=float, default=900.0)
    ap.add_argument("--ts-sample", type=float, default=30.0)
    ap.add_argument("--ts-seed", type=int, default=1)
    ap.add_argument("--accuracy-study", action="store_true",
                    help="split the DOS error of Ising runs into piece shape and join parts (exact DOS)")
    ap.add_argument("--acc-L", type=int, default=32)
    ap.add_argument("--acc-h", type=int, default=8)
    ap.add_argument("--acc-m", type=int, default=16)
    ap.add_argument("--acc-kfinal", type=int, default=20)
    ap.add_argument("--acc-seeds", type=int, default=4)
    ap.add_argument("--ensemble-study", action="store_true",
                    help="the paper's Potts L=100 workload as n runs + bootstrap + specific heat")
    ap.add_argument("--ens-runs", type=int, default=4)
    ap.add_argument("--ens-kfinal", type=int, default=10)
    ap.add_argument("--ens-R", type=int, default=200)
    ap.add_argument("--ens-tmin", type=float, default=0.68)
    ap.add_argument("--ens-tmax", type=float, default=0.74)
    ap.add_argument("--ens-nT", type=int, default=601)
    ap.add_argument("--ens-h", type=int, default=0, help="--ensemble-study: number of windows (0: 77)")
    ap.add_argument("--ens-windows", default="equal", choices=["equal", "ground-tilt"])
    ap.add_argument("--warm", action="store_true",
                    help="train the DOS network on REWL results of small systems and compare "
                         "time to converge, warm start against plain REWL, on larger targets")
    ap.add_argument("--train-kfinal", type=int, default=16)
    ap.add_argument("--train-types", default="small", choices=["tiny", "small", "batch"],
                    help="--warm: training instances (tiny: L 8 and 12; small: L <= 32/24; batch: the "
                         "batch's types, L <= 48)")
    ap.add_argument("--warm-seeds", type=int, default=1)
    ap.add_argument("--warm-targets", default="potts32,ising48")
    ap.add_argument("--warm-modes", default="warm,plain")
    ap.add_argument("--kfinal", type=int, default=18, help="--warm: targets' final ln f = 2^-kfinal")
    ap.add_argument("--k0", type=int, default=10,
                    help="--warm: warm start's initial ln f = 2^-k0 (-1: from the network's error)")
    ap.add_argument("--mlp-steps", type=int, default=4000)
    ap.add_argument("--target-seconds", type=float, default=200.0)
    args = ap.parse_args(argv)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); the multi-GPU layout is "
              "described, not built.", file=sys.stderr)
        return 2

    import paper_1407_5140_amd as rw

    if args.calib_copy_mib:
        import torch
        n = args.calib_copy_mib << 20
        src = torch.ones(n // 4, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        print(f"[bench] calibration copy of {args.calib_copy_mib} MiB done", file=sys.stderr, flush=True)
        return 0

    if args.warm:
        print(json.dumps(warm_start_study(rw, args)), flush=True)
        return 0
    if args.mlp_bench:
        print(json.dumps(mlp_bench(rw, args)), flush=True)
        return 0
    if args.warm_error_study:
        print(json.dumps(warm_error_study(rw, args)), flush=True)
        return 0
    if args.exchange_study:
        print(json.dumps(exchange_study(rw, args)), flush=True)
        return 0
    if args.ensemble_study:
        print(json.dumps(ensemble_study(rw, args)), flush=True)
        return 0
    if args.target_study:
        print(json.dumps(target_study(rw, args)), flush=True)
        return 0
    if args.accuracy_study:
        print(json.dumps(accuracy_study(rw, args)), flush=True)
        return 0
    if args.headline:
        print(json.dumps(headline_study(rw, args)), flush=True)
        return 0
    if args.balanced_study:
        print(json.dumps(balanced_study(rw, args)), flush=True)
        return 0
    kws = workload(args.workload)
    label = LABELS[args.workload]
    if args.converge:
        tune = rw.make_tune(args.sweep, args.wpb, 1, 200, table_placement=args.placement)
        kw = dict(kws[0], flat_rule=args.flat_rule)
        if args.flat:
            kw["flat"] = tuple(int(v) for v in args.flat.split(","))
        if args.m:
            kw["m"] = args.m
        if args.kfinal_override:
            kw["kfinal"] = args.kfinal_override
        if args.windows != "equal":
            kw["windows"] = tilted_windows(rw, kw)
        label += f"; flatness {kw['flat_rule']} {kw.get('flat', (4, 5))}, m={kw['m']}, kfinal={kw['kfinal']}"
        if args.windows != "equal":
            label += f"; windows {args.windows} {(kw['windows'][1] - kw['windows'][0] + 1).tolist()}"
        for sd in [int(x) for x in args.seeds.split(",")]:
            print(json.dumps(converge(rw, kw, label, tune, args.max_seconds, sd)), flush=True)
        return 0
    cfgs = [rw.make_config(**kw) for kw in kws]
    S = sum(kw["n_windows"] * kw["m"] for kw in kws)
    att_step = sum(kw["n_windows"] * kw["m"] * kw["X"] for kw in kws)
    t_create = time.perf_counter()
    # the timed steps replay the interval's captured HIP graph (no host work between
    # intervals); the kernel times come from a second pass of the same length with
    # per-launch events, which synchronises the host once per interval
    tune = rw.make_tune(args.sweep, args.wpb, 1, 1 << 20, lds_target_kb=args.lds_kb,
                        autotune=1 if args.autotune else 0, table_placement=args.placement,
                        persistent=1 if args.persistent else 0, map_log2=args.map_log2)
    g = rw.Rewl(cfgs, tune=tune)
    t_create = time.perf_counter() - t_create
    info = g.info()
    print(f"[bench] {label}: {S} walkers, {info['sweep_kind']} sweep ({info['table_placement']} counts, "
          f"{info['map_entries']} map entries), "
          f"walkers/block {info['walkers_per_block']}, "
          f"LDS {info['lds_bytes']} B, tune {g.tune()}, create {t_create:.2f} s", file=sys.stderr, flush=True)

    rw.rewl_run_exact(g.h, args.warmup)
    _sync()
    t0 = time.perf_counter()
    rw.rewl_run_exact(g.h, args.steps)
    _sync()
    dt = time.perf_counter() - t0
    rw.rewl_set_timing(g.h, True)
    st0 = g.stats()
    rw.rewl_run_exact(g.h, args.steps)
    st1 = g.stats()
    rw.rewl_set_timing(g.h, False)
    attempts = args.steps * att_step
    value = attempts / dt
    sweep_ms = (st1["sweep_ms"] - st0["sweep_ms"]) / args.steps
    interval_ms = (st1["interval_ms"] - st0["interval_ms"]) / args.steps
    ops = sum(OPS_PER_ATTEMPT[kw["model"]] * kw["n_windows"] * kw["m"] * kw["X"] for kw in kws)
    kernel = sweep_kernel(info, g.tune())
    traffic = profiled_traffic(args.workload, kernel)
    achieved = ops / (sweep_ms * 1e-3)
    print(f"[bench] {args.steps} intervals in {dt:.3f} s: {value:.4g} attempts/s; sweep "
          f"{sweep_ms:.3f} ms/launch, interval {interval_ms:.3f} ms (events)", file=sys.stderr,
          flush=True)

    out = {
        "metric": "spin-flip attempts/s; time to ln f=1e-8, MLP warm-start vs plain REWL",
        "value": value,
        "unit": "attempts/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": dt * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": label, "walkers": S, "attempts_per_step": att_step, "graph": True,
                   "sweep": info["sweep_kind"], "walkers_per_block": info["walkers_per_block"],
                   "table_placement": info["table_placement"], "map_entries": info["map_entries"]},
        "roofline": {"bound": "alu", "achieved": achieved / 1e12, "peak": PEAK_LANE_OPS / 1e12,
                     "unit": "Tops/s", "frac": achieved / PEAK_LANE_OPS,
                     "traffic": None if traffic is None else sum(traffic),
                     "traffic_read_write": traffic,
                     "kernel": kernel,
                     "kernel_ms": sweep_ms,
                     "ops_per_attempt": ops / att_step},
        "sweep_attempts_per_s": att_step / (sweep_ms * 1e-3),
    }
    g.close()
    if args.workload == "ising64" and not args.no_extras and not args.autotune:
        out["batch64"] = batch_line(rw)
        out["time_to_converge"] = ising8_converge(rw)
        out["warm_vs_plain"] = warm_line(rw)
    if not args.no_cpu_baseline:
        print("[bench] timing the oracle on the host cores", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(kws, args.cpu_budget)
    print(json.dumps(out), flush=True)
    return 0


def batch_line(rw, steps: int = 10, warmup: int = 2) -> dict:
    """The 64-instance batch, autotuned, timed like the main workload (extra keys)."""
    kws = workload("batch64")
    t0 = time.perf_counter()
    g = rw.Rewl([rw.make_config(**kw) for kw in kws],
                tune=rw.make_tune(autotune=1, use_graph=1, poll_every=1 << 20))
    t_create = time.perf_counter() - t0
    rw.rewl_run_exact(g.h, warmup)
    t0 = time.perf_counter()
    rw.rewl_run_exact(g.h, steps)                  # graph replays
    dt = time.perf_counter() - t0
    rw.rewl_set_timing(g.h, True)
    st0 = g.stats()
    rw.rewl_run_exact(g.h, steps)                  # per-launch events
    st1 = g.stats()
    att = steps * sum(kw["n_windows"] * kw["m"] * kw["X"] for kw in kws)
    ops = steps * sum(OPS_PER_ATTEMPT[kw["model"]] * kw["n_windows"] * kw["m"] * kw["X"] for kw in kws)
    sweep_ms = (st1["sweep_ms"] - st0["sweep_ms"]) / steps
    interval_ms = (st1["interval_ms"] - st0["interval_ms"]) / steps
    info, tune = g.info(), g.tune()
    g.close()
    kernel = sweep_kernel(info, tune)
    traffic = profiled_traffic("batch64", kernel)
    print(f"[bench] batch64: {att / dt:.4g} attempts/s, sweep {sweep_ms:.3f} ms/launch, interval "
          f"{interval_ms:.3f} ms, tune {tune}, create+autotune {t_create:.2f} s", file=sys.stderr, flush=True)
    return {"workload": LABELS["batch64"], "attempts_per_s": att / dt, "ms_per_step": dt * 1e3 / steps,
            "steps": steps, "sweep_ms": sweep_ms, "interval_ms": interval_ms, "graph": bool(tune["use_graph"]),
            "sweep": info["sweep_kind"], "lds_target_kb": tune["lds_target_kb"],
            "roofline": {"bound": "alu", "achieved": ops / steps / (sweep_ms * 1e-3) / 1e12,
                         "peak": PEAK_LANE_OPS / 1e12, "unit": "Tops/s",
                         "frac": ops / steps / (sweep_ms * 1e-3) / PEAK_LANE_OPS,
                         "traffic": None if traffic is None else sum(traffic),
                         "traffic_read_write": traffic, "kernel": kernel,
                         "persistent": bool(tune["persistent"])}}


def ising8_converge(rw, seeds=(1, 2, 3)) -> dict:
    """Time to converge of the Ising L=8 workload (4 windows, one walker each, ln f 1 ->
    2^-20 <= 1e-6), seeds run one after another, with the DOS error against the exact DOS."""
    from paper_1407_5140_amd import workloads as W
    kw0 = W.single("ising8")
    res = [converge(rw, kw0, LABELS["ising8"], rw.make_tune(poll_every=25), 60.0, sd) for sd in seeds]
    return {"workload": LABELS["ising8"], "seeds": list(seeds),
            "seconds": [r["seconds"] for r in res], "intervals": [r["intervals"] for r in res],
            "converged": [r["converged"] for r in res],
            "eps_mean": [r.get("eps_mean") for r in res], "eps_max": [r.get("eps_max") for r in res]}


def warm_line(rw, seeds=(1, 2, 3), k0: int = 8) -> dict:
    """The network's warm start against plain REWL, small enough for every bench run:
    the network is trained on REWL's own results (4 windows, 8 walkers, ln f -> 2^-13)
    for Ising L 8-16 and Potts q 4/8/10 L 8-12, produced here; the target is 10-state
    Potts L=16 (4 windows x 8 walkers, X = 2000) to ln f = 2^-13, three seeds warm (from
    2^-k0) and three plain (from 1), each group in its own handle.  Intervals are exactly
    reproducible (counter-based random numbers); seconds are the group's wall time."""
    from paper_1407_5140_amd import warm as Wm
    types = [("ising", 2, 8), ("ising", 2, 12), ("ising", 2, 16), ("potts", 4, 8), ("potts", 4, 12),
             ("potts", 8, 8), ("potts", 8, 12), ("potts", 10, 8), ("potts", 10, 12)]
    t0 = time.perf_counter()
    kws = Wm.training_workload(types, m=8, kfinal=13, X=2000, seed0=500)
    for kw in kws:
        kw["n_windows"] = 4
    g, res = Wm.run_to_convergence(kws, 120.0)
    ok = [r["converged"] for r in res]
    x, t = Wm.training_rows(g, kws, ok)
    g.close()
    net, info = Wm.train(x, t, steps=1500, batch=1024, lr=1e-3, seed=1)
    t_train = time.perf_counter() - t0
    base = dict(model="potts", q=10, L=16, n_windows=4, m=8, kfinal=13, X=2000)
    table = Wm.warm_table(net, base)
    net.close()
    out = {"workload": "10-state Potts L=16 periodic, 4 windows o=3/4, 8 walkers/window, X=2000, "
                       f"ln f 1 (plain) or 2^-{k0} (warm) -> 2^-13",
           "train": {"instances": len(kws), "converged": int(sum(ok)), "rows": int(len(t)),
                     "seconds_with_training": t_train, "rms": info["rms"]}}
    for mode in ("plain", "warm"):
        kk = [dict(base, seed=sd, k0=k0 if mode == "warm" else 0) for sd in seeds]
        ts = time.perf_counter()
        gg, rr = Wm.run_to_convergence(kk, 120.0, warm_tables=[table] * len(kk) if mode == "warm" else None,
                                       poll=10)
        wall = time.perf_counter() - ts
        gg.close()
        out[mode] = {"intervals": [r["intervals"] for r in rr], "converged": [r["converged"] for r in rr],
                     "seconds": wall}
    if all(out["plain"]["converged"]) and all(out["warm"]["converged"]):
        out["intervals_plain_over_warm"] = float(np.median(out["plain"]["intervals"]) /
                                                 np.median(out["warm"]["intervals"]))
        out["seconds_plain_over_warm"] = out["plain"]["seconds"] / out["warm"]["seconds"]
    print(f"[bench] warm vs plain: {out.get('intervals_plain_over_warm')} x fewer intervals, "
          f"{out.get('seconds_plain_over_warm')} x less time", file=sys.stderr, flush=True)
    return out


if __name__ == "__main__":
    sys.exit(main())
