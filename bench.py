"""Benchmark of the SU(2) heat-bath sweep on one MI355X.

Workload (default): 64^4 periodic lattice (1.07 GB of FP32 links), beta = 2.4,
hot start from Philox seed 1, plain Kennedy-Pendleton heat-bath -- the lattice
on which the HBM-roofline fraction is quoted.  The chain is first brought to
equilibrium (--therm sweeps, untimed).  One step = one measured configuration
of the paper's statistics run (Sec. 2.4: configurations 5 sweeps apart): five
full sweeps (eight (parity, mu) passes each), the last of which also sums the
plaquette in its even passes, then the plaquette reduction and the Polyakov
loop into a device-resident history -- every row of the hot path after
initialisation.  Inputs (the initialised lattice) are resident in HBM before
the timed region starts.

Prints one JSON line: throughput in link updates/s, the roofline of the
dominant kernel (k_pass, measured with HIP events on the library's stream
inside the timed region), and the CPU oracle timed on a bounded sample of the
same workload.
"""
import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "SU(2) link updates/s + HBM GB/s fraction; learned vs KP proposal at same <P>"
HBM_PEAK_GBS = 8000.0
BYTES_PER_UPDATE = 128  # one lattice streamed per (parity, mu) pass: 4N links x 16 B / (N/2) updates
# plan: the pass-kernel launch plan (tile order, LDS bytes) that su2_tune picks
# for the workload in most runs (its candidates within ~2 % of each other trade
# places from run to run); --tune re-tunes instead.  A fixed plan keeps the
# committed traffic counters (taken with that plan) applicable.
WORKLOADS = {
    64: dict(name="su2_64x64x64x64_b2.4_hot", dims=(64, 64, 64, 64), beta=2.4, seed=1, start=1,
             plan=(1108, 32768)),
    32: dict(name="su2_32x32x32x32_b2.3_hot", dims=(32, 32, 32, 32), beta=2.3, seed=1, start=1,
             plan=None),
}
FUSED_PAIRS = 300  # the launch plan that runs each parity as two fused-pair launches
SWEEPS_PER_STEP = 5  # Sec. 2.4: measured configurations are 5 sweeps apart
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_pass_traffic.json")
# everything the pass kernel is compiled from, and the build flags
KERNEL_SOURCES = [os.path.join(ROOT, "paper_0903_3053_amd", "csrc", f)
                  for f in ("su2_kernels.hip", "su2_kernels.hpp", "su2_device.hpp", "su2_pass.hpp",
                            "su2_pair.hpp")] + [os.path.join(ROOT, "paper_0903_3053_amd", "build.py")]


def kernel_hash():
    """Hash of the pass kernel's sources and build flags with comments and
    blank space taken out, so that a stored counter run stays valid across
    edits of comments only."""
    import re
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(f, "r") as fh:
            text = fh.read()
        if f.endswith(".py"):
            text = re.sub(r"#[^\n]*", "", text)
        else:
            text = re.sub(r"/\*.*?\*/", "", re.sub(r"//[^\n]*", "", text), flags=re.S)
        h.update(re.sub(r"\s+", " ", text).strip().encode())
    return h.hexdigest()[:16]


def measured_traffic(workload, plan):
    """HBM bytes per k_pass launch from the committed rocprofv3 counter runs,
    or None if they were taken on another version of the kernel or with
    another launch plan."""
    try:
        with open(TRAFFIC_FILE) as fh:
            t = json.load(fh)
    except (OSError, ValueError):
        return None
    rec = t.get(workload)
    if not rec or rec.get("kernel_hash") != kernel_hash() or list(rec.get("plan", [])) != list(plan):
        return None
    return rec.get("bytes_per_launch")


def cpu_model():
    """The host CPU's model name and logical core count (this process's affinity)."""
    name = "unknown"
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    name = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return name, len(os.sched_getaffinity(0))


def replica_check(replicas, gpu_hist, sweeps=300, cut=100):
    """The batched-replica workload's per-replica plaquette against the oracle:
    each listed replica (same extents, beta, seed, hot start) run by the oracle
    for `sweeps` sweeps, <P> over the sweeps after `cut`, against the GPU's
    <P> over its recorded equilibrium history of the same replica; both errors
    by the Gamma method."""
    import numpy as np
    import oracle
    from paper_0903_3053_amd.stats import gamma_method
    rows = []
    t0 = time.perf_counter()
    for r, h in zip(replicas, gpu_hist):
        ch = oracle.Chain(r["dims"], r["beta"], r["seed"], oracle.HOT)
        ph = []
        for _ in range(sweeps):
            ch.sweep(1)
            ph.append(ch.plaquette()[0])
        mo, eo, to, _, _ = gamma_method(np.asarray(ph[cut:]))
        mg, eg, tg, _, _ = gamma_method(np.asarray(h))
        rows.append({"replica": r["index"], "L": r["dims"][0], "beta": r["beta"],
                     "gpu": {"plaquette": mg, "err": eg, "sweeps": len(h)},
                     "oracle": {"plaquette": mo, "err": eo, "sweeps": sweeps - cut},
                     "z": (mg - mo) / float(np.hypot(eg, eo))})
    return {"replicas": rows, "max_abs_z": max(abs(x["z"]) for x in rows) if rows else None,
            "oracle_seconds": time.perf_counter() - t0}


def cpu_baseline(w, sweeps=8):
    """The oracle (plain C, FP64, OpenMP over sites) on a bounded sample of the
    same workload: the first `sweeps` sweeps of the same lattice from the same
    hot start (initialisation not timed) on every host thread, then the next
    pass (odd sites, mu = 0) on one thread."""
    import ctypes
    import oracle
    U = oracle.init(w["dims"], w["seed"], oracle.HOT)
    t0 = time.perf_counter()
    for s in range(sweeps):
        oracle.sweep(w["dims"], U, w["beta"], w["seed"], s)
    dt = time.perf_counter() - t0
    n = 4 * U.shape[0] * sweeps
    cores = oracle.num_threads()
    # the oracle's OpenMP runtime (libgomp, already loaded with it)
    gomp = ctypes.CDLL("libgomp.so.1")
    gomp.omp_set_num_threads(1)
    t1 = time.perf_counter()
    oracle.heatbath_pass(w["dims"], U, w["beta"], w["seed"], sweeps, 1, 0)
    dt1 = time.perf_counter() - t1
    gomp.omp_set_num_threads(cores)
    n1 = U.shape[0] // 2
    del U
    model, host_cores = cpu_model()
    return {"value": n / dt, "unit": "link updates/s", "cores": cores,
            "kind": "oracle", "cpu_model": model, "host_logical_cores": host_cores,
            "sample": f"the first {sweeps} sweeps ({n} link updates) of the same {w['name']} "
                      f"lattice from the same hot start, {dt:.2f} s wall",
            "single_thread": {"value": n1 / dt1, "unit": "link updates/s", "cores": 1,
                              "sample": f"the next pass (odd sites, mu = 0: {n1} link updates), "
                                        f"{dt1:.2f} s wall"}}


def batched_replicas(su2, sweeps=500, compare_sweeps=50):
    """The batched-replica workload: 64 lattices, L uniform on {8, 12, 16, 20,
    24}, beta uniform on [1.8, 2.8], hot starts from per-replica seeds, `sweeps`
    sweeps of every replica in the tuned launch mode; also the grouped mode and
    the persistent mode (8 tiles per work item) timed side by side."""
    import numpy as np
    import torch
    import su2_inputs
    table = su2_inputs.replica_table(64, 1)
    dims = [t["dims"] for t in table]
    V = sum(int(np.prod(d)) for d in dims)
    su2.su2_batch_init(dims, [t["beta"] for t in table], [t["seed"] for t in table], 1)
    modes = {}
    for name, mode in (("grouped", (0, 1, 0)), ("persistent", (1, 8, 0))):
        su2.su2_batch_set_mode(*mode)
        su2.su2_batch_sweep(2)  # build the graph, warm up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su2.su2_batch_sweep(compare_sweeps)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        modes[name] = 4 * V * compare_sweeps / dt
    su2.su2_batch_init(dims, [t["beta"] for t in table], [t["seed"] for t in table], 1)
    # a persistent launch pays its start and drain once per call: time candidates
    # over enough sweeps per call for that to amortise as in the run below
    chosen = su2.su2_batch_tune(20)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    su2.su2_batch_sweep(sweeps)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    P = su2.su2_batch_plaquette()
    # per-replica plaquette histories at equilibrium (after the timed sweeps),
    # for the comparison with the oracle's chains of the same replicas
    check = [dict(t, index=r) for r, t in enumerate(table) if t["dims"][0] == 8][:CHECK_REPLICAS]
    hist = [[] for _ in check]
    for _ in range(CHECK_SWEEPS):
        su2.su2_batch_sweep(1)
        Pr = su2.su2_batch_plaquette()
        for j, c in enumerate(check):
            hist[j].append(float(Pr[c["index"], 0]))
    su2.su2_batch_finalize()
    upd = 4 * V * sweeps
    return {"workload": "64 replicas, L uniform on {8,12,16,20,24}, beta uniform on [1.8,2.8], hot, "
                        f"{sweeps} sweeps", "sites": V, "value": upd / dt, "unit": "link updates/s",
            "seconds": dt, "algorithmic_GBps": upd * BYTES_PER_UPDATE / dt / 1e9,
            "algorithmic_frac": upd * BYTES_PER_UPDATE / dt / 1e9 / HBM_PEAK_GBS,
            "_check": (check, hist),
            "mode": {"persistent": bool(chosen[0]), "tiles_per_item": chosen[1], "lds_bytes": chosen[2]},
            "updates_per_s_by_mode": modes,
            "plaquette_range": [float(P[:, 0].min()), float(P[:, 0].max())]}


CHECK_REPLICAS = 4   # replicas whose plaquette the cpu_baseline leg compares with the oracle
CHECK_SWEEPS = 200   # recorded sweeps of each
TABLE_ROWS = 31


def learned_proposal(su2, sweeps=100000, train_steps=30000):
    """The learned-proposal workload: the network trained on the device on the
    integrated CDFs of 4096 alphas, then 32^4 beta = 2.3 from the same hot start
    for `sweeps` sweeps with the heat-bath, with the learned independence-
    Metropolis step, and with the same step reading the integrated CDF's knots
    instead of the network's (the ablation: what the network's approximation
    costs); plaquette measured every sweep, averages after a 10 %
    thermalisation cut with Gamma-method errors and integrated autocorrelation
    times; updates/s of the three from interleaved timing rounds."""
    import numpy as np
    import torch
    import su2_inputs
    from paper_0903_3053_amd.stats import gamma_method
    dims, beta, seed = (32, 32, 32, 32), 2.3, 1
    V = int(np.prod(dims))
    su2.su2_mlp_set_params(su2_inputs.mlp_init(1))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hist = su2.su2_mlp_train(su2_inputs.alpha_grid(4096), train_steps, 3e-3, 1e-5)
    # the sweep reads a knot table of TABLE_ROWS alphas on [0, 40] (linear in
    # alpha between rows); 31 rows fit the pass kernel's LDS copy
    su2.su2_mlp_tabulate(TABLE_ROWS)
    t_train = time.perf_counter() - t0

    chains = (("kennedy_pendleton", 0, None), ("learned_imh", 1, su2.su2_mlp_tabulate),
              ("exact_knots_imh", 1, su2.su2_cdf_tabulate))

    def use(kind, table, plan=None):
        if table is not None:
            table(TABLE_ROWS)
        if plan is not None:
            su2.su2_set_plan(*plan)
        su2.su2_set_proposal(kind)

    out = {}
    plans = {}
    for name, kind, table in chains:
        # each proposal runs with the launch plan tuned for it
        su2.su2_init(dims, beta, seed, 1)
        use(kind, table)
        su2.su2_sweep(5)
        plans[name] = su2.su2_tune(2)
        su2.su2_init(dims, beta, seed, 1)
        use(kind, table, plans[name])
        h = su2.su2_sweep_measure(sweeps, 1)[:, 0]
        m, e, tau, dtau, _ = gamma_method(h[sweeps // 10:])
        rec = {"plaquette": m, "plaquette_err": e, "tau_int_sweeps": tau, "tau_int_err": dtau,
               "sweeps_analysed": sweeps - sweeps // 10,
               "pass_plan": {"tile_order": plans[name][0], "lds_bytes": plans[name][1]}}
        if kind:
            prop, acc = su2.su2_imh_counters()
            rec["acceptance"] = acc / max(prop, 1)
        out[name] = rec
    # rates: TIMING_ROUNDS rounds cycling through the three on the same
    # equilibrated chain (200 sweeps each, after 2 untimed sweeps that build
    # the graphs of the switched plan), so clock or cache drifts hit all alike;
    # the median of each and of the per-round ratios is reported
    su2.su2_init(dims, beta, seed, 1)
    su2.su2_sweep(200)
    rates = {name: [] for name, _, _ in chains}
    for _ in range(TIMING_ROUNDS):
        for name, kind, table in chains:
            use(kind, table, plans[name])
            su2.su2_sweep(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            su2.su2_sweep(200)
            torch.cuda.synchronize()
            rates[name].append(4 * V * 200 / (time.perf_counter() - t0))
    for name, _, _ in chains:
        out[name]["link_updates_per_s"] = float(np.median(rates[name]))
        out[name]["link_updates_per_s_rounds"] = rates[name]
    kp = out["kennedy_pendleton"]
    for name in ("learned_imh", "exact_knots_imh"):
        r = out[name]
        ratios = [b / a for a, b in zip(rates["kennedy_pendleton"], rates[name])]
        r["speed_ratio"] = float(np.median(ratios))
        r["speed_ratio_rounds"] = ratios
        # updates/s per integrated autocorrelation time of <P>: independent
        # samples/s, relative to the heat-bath; the error from the two tau_int
        eff = r["speed_ratio"] * kp["tau_int_sweeps"] / r["tau_int_sweeps"]
        r["effective_speed_ratio"] = eff
        r["effective_speed_ratio_err"] = eff * float(np.hypot(kp["tau_int_err"] / kp["tau_int_sweeps"],
                                                              r["tau_int_err"] / r["tau_int_sweeps"]))
        r["z_plaquette_vs_heat_bath"] = (r["plaquette"] - kp["plaquette"]) / float(
            np.hypot(kp["plaquette_err"], r["plaquette_err"]))
    # what training buys: the same step on the untrained network's table and
    # on uniform knots (all parameters zero: equal softmax widths), shorter
    # chains, rates timed beside the heat-bath's on the learned plan
    trained, _ = su2.su2_mlp_get_params()
    ablations = {}
    for name, params in (("untrained_imh", su2_inputs.mlp_init(1)),
                         ("uniform_knots_imh", np.zeros_like(trained))):
        su2.su2_mlp_set_params(params)
        su2.su2_mlp_tabulate(TABLE_ROWS)
        su2.su2_init(dims, beta, seed, 1)
        use(1, None, plans["learned_imh"])
        n_ab = max(sweeps // 5, 1000)
        h = su2.su2_sweep_measure(n_ab, 1)[:, 0]
        prop, acc = su2.su2_imh_counters()
        m, e, tau, dtau, _ = gamma_method(h[n_ab // 10:])
        t = {}
        for kind in (0, 1):
            use(kind, None, plans["learned_imh"])
            su2.su2_sweep(2)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            su2.su2_sweep(200)
            torch.cuda.synchronize()
            t[kind] = 4 * V * 200 / (time.perf_counter() - t0)
        ablations[name] = {"acceptance": acc / max(prop, 1), "sweeps": n_ab, "plaquette": m, "plaquette_err": e,
                           "tau_int_sweeps": tau, "tau_int_err": dtau, "link_updates_per_s": t[1],
                           "heat_bath_link_updates_per_s_same_plan": t[0],
                           "effective_speed_ratio": (t[1] / tau) / (t[0] / kp["tau_int_sweeps"])}
    su2.su2_mlp_set_params(trained)
    su2.su2_mlp_tabulate(TABLE_ROWS)
    scan = beta_scan(su2, dims, seed, {0: plans["kennedy_pendleton"], 1: plans["learned_imh"]})
    su2.su2_finalize()
    lp = out["learned_imh"]
    return {"workload": f"32^4 beta 2.3 hot seed 1, {sweeps} sweeps each: heat-bath, learned proposal, "
                        f"and the same proposal on the integrated CDF's knots",
            "beta_scan": scan,
            "ablations": ablations,
            "training": {"steps": train_steps, "alphas": 4096, "seconds": t_train, "table_rows": TABLE_ROWS,
                         "loss_first": float(hist[0]), "loss_last": float(hist[-1])},
            **out,
            "z_plaquette": lp["z_plaquette_vs_heat_bath"],
            "speed_ratio": lp["speed_ratio"],
            "effective_speed_ratio": lp["effective_speed_ratio"],
            "effective_speed_ratio_err": lp["effective_speed_ratio_err"]}


def couplings_32(su2, sweeps=1000, cut=200):
    """The 32^4 workload as configured (hot start, Philox seed 1, plain
    heat-bath, 1000 sweeps, the plaquette reduced in FP64 after every sweep)
    at beta in {2.2, 2.3, 2.4, 2.5}, each with the tuned launch plan: the
    sweeps from the hot start with the history kept on the device
    (su2_sweep_measure), timed on the library's stream, the statistics of the
    plaquette after `cut` sweeps; then as many sweeps without measurement,
    timed alike.  The lattice (64 MiB) fits the 256 MB Infinity Cache, so the
    bytes fraction is of the algorithmic traffic, not a measure of HBM."""
    import numpy as np
    import torch
    from paper_0903_3053_amd.stats import gamma_method
    w = su2_inputs_workload("su2_32x32x32x32_hot")
    dims = w["dims"]
    V = int(np.prod(dims))
    rows = []
    for beta in w["betas"]:
        su2.su2_init(dims, beta, w["seed"], w["start"])
        plan = su2.su2_tune(2)
        su2.su2_init(dims, beta, w["seed"], w["start"])  # the tuner swept; start again
        su2.su2_set_plan(*plan)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        h = su2.su2_sweep_measure(sweeps, 1)
        dt = time.perf_counter() - t0
        rate = 4 * V * sweeps / dt
        # the sweeps alone (no measurement), on the library's stream
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su2.su2_sweep(sweeps)
        torch.cuda.synchronize()
        rate_sweeps = 4 * V * sweeps / (time.perf_counter() - t0)
        m, e, tau, _, _ = gamma_method(h[cut:, 0])
        rows.append({"beta": beta, "link_updates_per_s": rate,
                     "algorithmic_GBps": rate * BYTES_PER_UPDATE / 1e9,
                     "algorithmic_frac": rate * BYTES_PER_UPDATE / 1e9 / HBM_PEAK_GBS,
                     "sweeps_only_link_updates_per_s": rate_sweeps,
                     "sweeps_only_algorithmic_frac": rate_sweeps * BYTES_PER_UPDATE / 1e9 / HBM_PEAK_GBS,
                     "plaquette": m, "plaquette_err": e, "tau_int_sweeps": tau,
                     "pass_plan": {"tile_order": plan[0], "lds_bytes": plan[1]}})
    su2.su2_finalize()
    return {"workload": f"32^4 hot seed {w['seed']}, {sweeps} sweeps from the hot start with the plaquette "
                        f"after every sweep (statistics after sweep {cut}), then {sweeps} unmeasured",
            "points": rows}


def su2_inputs_workload(name):
    import su2_inputs
    return su2_inputs.WORKLOADS[name]


SCAN_BETAS = (0.5, 1.0, 1.5, 2.0, 2.3, 2.8)
TIMING_ROUNDS = 5


def beta_scan(su2, dims, seed, plans, therm=20, sweeps=100):
    """Both proposals over a range of couplings on the same lattice, each with
    its launch plan: updates/s over `sweeps` sweeps after `therm` sweeps from
    the hot start, heat-bath attempts and cap failures per update, and the
    learned proposal's acceptance.  At small beta*|staple| the heat-bath's
    rejection loop is long and a wavefront runs until its slowest lane has
    accepted (or hit the cap of 8 attempts)."""
    import numpy as np
    import torch
    V = int(np.prod(dims))
    upd = 4 * V * sweeps
    rows = []
    for beta in SCAN_BETAS:
        rec = {"beta": beta}
        for name, kind in (("kennedy_pendleton", 0), ("learned_imh", 1)):
            su2.su2_init(dims, beta, seed, 1)
            su2.su2_set_plan(*plans[kind])
            su2.su2_set_proposal(kind)
            su2.su2_sweep(therm)
            a0, f0 = su2.su2_counters()[:2]
            p0, c0 = su2.su2_imh_counters()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            su2.su2_sweep(sweeps)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            a1, f1 = su2.su2_counters()[:2]
            r = {"link_updates_per_s": upd / dt, "plaquette": su2.su2_plaquette()}
            if kind:
                p1, c1 = su2.su2_imh_counters()
                r["acceptance"] = (c1 - c0) / max(p1 - p0, 1)
            else:
                r["attempts_per_update"] = (a1 - a0) / upd
                r["cap_failures_per_update"] = (f1 - f0) / upd
            rec[name] = r
        rec["speed_ratio"] = rec["learned_imh"]["link_updates_per_s"] / rec["kennedy_pendleton"]["link_updates_per_s"]
        rows.append(rec)
    return {"lattice": list(dims), "hot_start_seed": seed, "thermalisation_sweeps": therm,
            "timed_sweeps": sweeps, "points": rows}


def overrelaxation(su2, steps=500, n_or=3):
    """Overrelaxation sweeps (U -> V U^dag V about the staple direction): their
    rate on the 64^4 benchmark lattice (old link read: 144 B per update), and
    at 32^4 beta = 2.3 the plaquette's integrated autocorrelation time of the
    heat-bath chain against 1 heat-bath + n_or overrelaxation sweeps per step,
    each with the tuned launch plan, as the time per independent sample."""
    import numpy as np
    import torch
    from paper_0903_3053_amd.stats import gamma_method
    w = WORKLOADS[64]
    V64 = int(np.prod(w["dims"]))
    su2.su2_init(w["dims"], w["beta"], w["seed"], w["start"])
    su2.su2_set_plan(*w["plan"])
    su2.su2_sweep(1)
    su2.su2_overrelax(2)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    su2.su2_overrelax(20)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    pass_ms = dt * 1e3 / (20 * 8)
    or_bytes = (V64 // 2) * (BYTES_PER_UPDATE + 16)
    rate64 = 4 * V64 * 20 / dt
    su2.su2_finalize()

    dims, beta, seed = (32, 32, 32, 32), 2.3, 1
    V = int(np.prod(dims))
    su2.su2_init(dims, beta, seed, 1)
    su2.su2_tune(2)
    su2.su2_sweep(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    hb = su2.su2_sweep_measure(steps, 1)[:, 0]
    t_hb = (time.perf_counter() - t0) / steps
    su2.su2_init(dims, beta, seed, 1)
    su2.su2_sweep(100)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(100):
        su2.su2_sweep(1)
        su2.su2_overrelax(n_or)
    torch.cuda.synchronize()
    t_mix = (time.perf_counter() - t0) / 100
    mix = []
    for _ in range(steps):
        su2.su2_sweep(1)
        su2.su2_overrelax(n_or)
        mix.append(su2.su2_plaquette())
    su2.su2_finalize()
    m0, e0, tau0, _, _ = gamma_method(hb)
    m1, e1, tau1, _, _ = gamma_method(np.asarray(mix))
    return {"sweep_rate_64x64x64x64": {"link_updates_per_s": rate64, "avg_pass_ms": pass_ms,
                                        "algorithmic_bytes_per_pass": or_bytes,
                                        "hbm_frac": or_bytes / (pass_ms * 1e-3) / 1e9 / HBM_PEAK_GBS},
            "chain_32x32x32x32_b2.3": {
                "heat_bath": {"plaquette": m0, "plaquette_err": e0, "tau_int_steps": tau0,
                              "ms_per_step": t_hb * 1e3},
                f"heat_bath_plus_{n_or}_overrelaxation": {"plaquette": m1, "plaquette_err": e1,
                                                          "tau_int_steps": tau1, "ms_per_step": t_mix * 1e3},
                "z_plaquette": (m1 - m0) / float(np.hypot(e0, e1)),
                # time per independent sample of <P>: ms per step x 2 tau_int
                "speedup_per_independent_sample": (t_hb * tau0) / (t_mix * tau1),
                "steps": steps}}


# Table 1 of the paper (ATI RV770 GPU seconds for its SU(2) runs on L_t x L_s^3)
TABLE1_GPU_SECONDS = {(4, 8): 5.2, (4, 16): 17.9, (4, 24): 52.8, (4, 32): 120.6,
                      (8, 16): 32.7, (8, 24): 102.3, (8, 32): 397.4}


def paper_table1(su2, therm=1000, meas=1000, every=5, beta=2.3):
    """The paper's own SU(2) geometries (Table 1), read as 1000 thermalisation
    sweeps and 1000 measurements 5 sweeps apart (6000 sweeps), hot start, each
    with its tuned launch plan (tuning not timed): wall seconds here beside the
    RV770 seconds the paper prints (context, not a target: the paper does not
    give beta or the exact sweep count)."""
    import numpy as np
    import torch
    out = []
    for (lt, ls), paper_s in TABLE1_GPU_SECONDS.items():
        dims = (ls, ls, ls, lt)  # mu = 3 is time
        su2.su2_init(dims, beta, 1, 1)
        plan = su2.su2_tune(2)  # on a copy of the links: the chain is untouched
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        su2.su2_sweep(therm)
        hist = su2.su2_sweep_measure(meas * every, every)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        out.append({"lattice": f"{lt}x{ls}^3", "seconds": dt, "paper_rv770_seconds": paper_s,
                    "pass_plan": {"tile_order": plan[0], "lds_bytes": plan[1]},
                    "ratio": paper_s / dt, "sweeps": therm + meas * every,
                    "plaquette": float(np.mean(hist[len(hist) // 5:, 0]))})
    su2.su2_finalize()
    return {"beta": beta, "reading": "1000 thermalisation sweeps + 1000 measurements 5 sweeps apart",
            "runs": out}


def strong_coupling(su2, therm=100, timed=200, meas=400, switch=1.6847376):
    """Small beta on 32^4, hot start: plain Kennedy-Pendleton against the
    heat-bath with Creutz's draw below alpha = switch (su2_set_creutz), each
    with its tuned launch plan: link updates/s, attempts and cap failures per
    update, <P> of the two chains against each other and, for beta <= 0.5
    (where the omitted O(u^9) terms are below 1e-6), beside the
    strong-coupling series u + 4 u^5, u = I2(beta) / I1(beta).  KP's
    acceptance collapses as alpha -> 0; capped updates keep their link."""
    import numpy as np
    import torch
    from scipy import special
    from paper_0903_3053_amd.stats import gamma_method
    dims = (32, 32, 32, 32)
    n_upd = 4 * int(np.prod(dims))
    out = {"lattice": "32x32x32x32", "switch": switch}
    for beta in (0.25, 0.5, 1.0):
        u = special.iv(2, beta) / special.iv(1, beta)
        row = {"series_plaquette": u + 4 * u ** 5 if beta <= 0.5 else None}
        for name, sw in (("kennedy_pendleton", 0.0), ("with_creutz_switch", switch)):
            su2.su2_init(dims, beta, 1, 1)
            su2.su2_set_creutz(sw)
            plan = su2.su2_tune(2)
            su2.su2_sweep(therm)
            c0 = su2.su2_counters()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            su2.su2_sweep(timed)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            c1 = su2.su2_counters()
            hist = su2.su2_sweep_measure(meas, 1)
            m, e, tau, _, _ = gamma_method(hist[:, 0])
            row[name] = {"link_updates_per_s": n_upd * timed / dt,
                         "attempts_per_update": (c1[0] - c0[0]) / (n_upd * timed),
                         "cap_failures_per_update": (c1[1] - c0[1]) / (n_upd * timed),
                         "plaquette": m, "plaquette_err": e,
                         "z_vs_series": (m - row["series_plaquette"]) / e if row["series_plaquette"] else None,
                         "pass_plan": {"tile_order": plan[0], "lds_bytes": plan[1]}}
        kp, cr = row["kennedy_pendleton"], row["with_creutz_switch"]
        row["speedup"] = cr["link_updates_per_s"] / kp["link_updates_per_s"]
        row["z_switch_vs_kp"] = (cr["plaquette"] - kp["plaquette"]) / float(np.hypot(kp["plaquette_err"],
                                                                                     cr["plaquette_err"]))
        out[f"beta_{beta}"] = row
    su2.su2_finalize()
    return out


def ising_2d():
    """The paper's other workload (Sec. 2.3): 2-D Ising Metropolis on a red-black
    partition, beta = 0.44 (near the critical point), hot start, on the paper's
    1024 x 512 lattice and on 16384^2, in both device layouts (a byte per spin;
    1-bit spins, 32 per word, the default where L0 % 64 == 0 and N >= 2^20); spin updates/s
    with the lattice resident on the device (both layouts run the same chain).
    Algorithmic bytes per spin update: 3 (bytes: own colour read and written,
    other colour read) or 3/8 (bits).  The paper quotes 630 s for 10^6 sweeps
    of 1024 x 512 on ATI RV770 (8.3e8 spin updates/s), as context only."""
    import torch
    from paper_0903_3053_amd import ising
    out = {}
    for dims, n in (((1024, 512), 2000), ((16384, 16384), 50)):
        row = {}
        for name, layout, bytes_per in (("bytes", ising.LAYOUT_BYTES, 3.0), ("bits", ising.LAYOUT_BITS, 0.375)):
            ising.ising_init(dims, 0.44, 1, 1, layout)
            ising.ising_sweep(10)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ising.ising_sweep(n)
            torch.cuda.synchronize()
            dt = time.perf_counter() - t0
            N = dims[0] * dims[1]
            e, m = ising.ising_observables()
            rate = N * n / dt
            row[name] = {"spin_updates_per_s": rate, "us_per_sweep": dt / n * 1e6, "sweeps": n,
                         "energy_per_site": e, "magnetisation": m,
                         "algorithmic_GBps": rate * bytes_per / 1e9}
        row["bits_over_bytes"] = row["bits"]["spin_updates_per_s"] / row["bytes"]["spin_updates_per_s"]
        out[f"{dims[0]}x{dims[1]}"] = row
    # the paper's statistics run: a measurement (energy, magnetisation, returned
    # to the host) after every sweep, on 1024 x 512 with the default layout
    ising.ising_init((1024, 512), 0.44, 1, 1)
    ising.ising_sweep(10)
    n = 500
    t0 = time.perf_counter()
    for _ in range(n):
        ising.ising_sweep(1)
        ising.ising_observables()
    dt = time.perf_counter() - t0
    out["1024x512_measured"] = {"us_per_sweep_and_measurement": dt / n * 1e6, "sweeps": n,
                                "paper_rv770_us": 730.0}
    ising.ising_finalize()
    out["paper_context"] = {"hardware": "ATI RV770", "lattice": "1024x512",
                            "seconds_per_1e6_sweeps": 630, "spin_updates_per_s": 524288 * 1e6 / 630}
    return out


def host_transfer(su2, V, updates, timed_ms, reps=3):
    """The links through host memory: su2_links (device -> host) and
    su2_set_links (host -> device, same values and sweep index, so the chain
    is unchanged) on the benchmark's lattice, each timed over reps calls after
    one untimed call; and the rate of a run that loads its configuration from
    host memory, takes the timed steps and reads the result back.  Context
    only: the bench value keeps the links resident in HBM."""
    import numpy as np
    s0 = su2.su2_sweep_index()
    U = su2.su2_links()
    t = time.perf_counter()
    for _ in range(reps):
        U = su2.su2_links()
    t_out = (time.perf_counter() - t) / reps
    su2.su2_set_links(U, s0)
    t = time.perf_counter()
    for _ in range(reps):
        su2.su2_set_links(U, s0)
    t_in = (time.perf_counter() - t) / reps
    assert np.array_equal(su2.su2_links(), U)
    nbytes = 64 * V
    return {"bytes": nbytes, "links_out_ms": t_out * 1e3, "links_in_ms": t_in * 1e3,
            "GBps_out": nbytes / t_out / 1e9, "GBps_in": nbytes / t_in / 1e9,
            "pcie_inclusive_link_updates_per_s": updates / (timed_ms / 1e3 + t_in + t_out),
            "note": "pageable numpy buffers through the library's staging copy; the timed steps with "
                    "one load from and one copy back to host memory added; not the bench value"}


EXTRAS = ("batched_replicas", "couplings_32x32x32x32", "learned_proposal", "overrelaxation",
          "strong_coupling", "ising_2d", "paper_table1")
EXTRA_FUNCS = {"batched_replicas": batched_replicas, "couplings_32x32x32x32": couplings_32,
               "learned_proposal": learned_proposal, "overrelaxation": overrelaxation,
               "strong_coupling": strong_coupling, "ising_2d": lambda su2: ising_2d(),
               "paper_table1": paper_table1}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--lattice", type=int, default=64, choices=sorted(WORKLOADS))
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the extra workloads (batched replicas, 32^4 couplings, learned "
                         "proposal, overrelaxation, strong coupling, Ising, Table-1 geometries)")
    ap.add_argument("--extra", action="append", choices=EXTRAS, default=None,
                    help="run only this extra workload (repeatable); default: all of them")
    ap.add_argument("--tune", action="store_true",
                    help="pick the pass-kernel launch plan with su2_tune instead of the workload's")
    ap.add_argument("--plan", type=int, nargs=2, metavar=("ORDER", "LDS"), default=None,
                    help="use this pass-kernel launch plan")
    ap.add_argument("--therm", type=int, default=300,
                    help="untimed sweeps after the hot start, before the warm-up steps")
    ap.add_argument("--learned-sweeps", type=int, default=100000,
                    help="sweeps of each chain in the learned-proposal workload")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="first run a plain 1 GiB device copy (torch), so that a counter "
                         "profile of this command also holds the copy of known size")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              "(replicas and couplings would shard with no communication)", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_0903_3053_amd import su2

    w = WORKLOADS[args.lattice]
    dims = w["dims"]
    V = int(np.prod(dims))
    torch.cuda.set_device(0)
    stream = torch.cuda.Stream()
    su2.su2_set_stream(stream)
    su2.su2_init(dims, w["beta"], w["seed"], w["start"])
    hist = torch.zeros((args.steps, 4), dtype=torch.float64, device="cuda")
    # the pass kernel's launch plan (tile order, LDS reservation): results do
    # not depend on it
    if args.copy_calibration:
        a = torch.ones(2**28, dtype=torch.float32, device="cuda")
        b = torch.empty_like(a)
        for _ in range(3):
            b.copy_(a)
        torch.cuda.synchronize()
        del a, b
    if args.plan is not None or (w["plan"] is not None and not args.tune):
        plan = tuple(args.plan if args.plan is not None else w["plan"])
        su2.su2_set_plan(*plan)
    else:
        plan = su2.su2_tune(2)

    # thermalisation, then warm-up steps: sweeps and measurements, graphs built
    # and replayed
    su2.su2_sweep(args.therm)
    for i in range(args.warmup):
        su2.su2_sweep_measured(SWEEPS_PER_STEP)
        su2.su2_measure_device(hist[i % args.steps])
    torch.cuda.synchronize()
    c_start = su2.su2_counters()

    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    start_ev = torch.cuda.Event(enable_timing=True)
    end_ev = torch.cuda.Event(enable_timing=True)
    start_ev.record(stream)
    for i in range(args.steps):
        ev[i][0].record(stream)
        # one graph: the step's sweeps and one sweep-index tick; the last
        # sweep's even passes also sum the plaquette
        su2.su2_sweep_measured(SWEEPS_PER_STEP)
        ev[i][1].record(stream)
        su2.su2_measure_device(hist[i])  # reduce those partials + Polyakov loop
    end_ev.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    total_ms = start_ev.elapsed_time(end_ev)
    sweep_ms = sum(a.elapsed_time(b) for a, b in ev)
    ms_per_step = max(total_ms, wall * 1e3) / args.steps
    c_end = su2.su2_counters()
    updates = 4 * V * SWEEPS_PER_STEP * args.steps
    value = updates / (ms_per_step * args.steps / 1e3)
    h = hist.cpu().numpy()
    P, poly = h[-1, :3], h[-1, 3]

    # roofline of the sweep kernel: k_pass, 8 launches per sweep of V/2 updates
    # x 128 B; or, with the fused-pair plan, k_pair, 4 launches of two passes each
    fused = plan[0] == FUSED_PAIRS
    launches = 4 if fused else 8
    pass_ms = sweep_ms / (launches * SWEEPS_PER_STEP * args.steps)
    bytes_per_launch = (8 // launches) * (V // 2) * BYTES_PER_UPDATE
    achieved = bytes_per_launch / (pass_ms * 1e-3) / 1e9
    traffic = None if fused else measured_traffic(w["name"], plan)
    # the whole step against the same roofline: its algorithmic bytes (the
    # sweeps' 128 B per update plus the Polyakov loop's 16 B per site; the
    # plaquette is summed from staples the sweep holds) over its wall time
    step_bytes = updates * BYTES_PER_UPDATE / args.steps + 16 * V
    step_gbs = step_bytes / (ms_per_step * 1e-3) / 1e9

    rec = {
        "metric": METRIC, "value": value, "unit": "link updates/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms_per_step,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w["name"], "dims": list(dims), "beta": w["beta"], "seed": w["seed"],
                   "start": "hot", "proposal": "kennedy-pendleton",
                   "step": f"one measured configuration (Sec. 2.4: 5 sweeps apart): {SWEEPS_PER_STEP} sweeps "
                           + ("(4 fused-pair launches each" if fused else "(8 passes each")
                           + ", the last sweep's even passes also summing the plaquette) + plaquette "
                             "reduction + Polyakov loop, on device, at equilibrium",
                   "thermalisation_sweeps": args.therm,
                   "pass_plan": {"tile_order": plan[0], "lds_bytes": plan[1]}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_source": ("stored rocprofv3 FETCH_SIZE + WRITE_SIZE runs (copy-calibrated) "
                                        "of this kernel source and plan, profiles/k_pass_traffic.json; "
                                        "not measured in this run") if traffic is not None else
                                       "none stored for this kernel source and plan",
                     "kernel": "k_pair" if fused else "k_pass", "avg_launch_ms": pass_ms,
                     "algorithmic_bytes_per_launch": bytes_per_launch,
                     "timing": "HIP events on the library's stream around each step's sweeps "
                               f"({launches * SWEEPS_PER_STEP} launches + one sweep-index tick, one graph)"},
        "roofline_step": {"achieved": step_gbs, "frac": step_gbs / HBM_PEAK_GBS, "unit": "GB/s",
                          "algorithmic_bytes_per_step": step_bytes,
                          "updates_frac": value * BYTES_PER_UPDATE / 1e9 / HBM_PEAK_GBS,
                          "note": "whole step on its wall clock: sweeps + reductions + Polyakov loop; "
                                  "updates_frac counts the sweeps' 128 B per update only"},
        "observables": {"plaquette": float(P[0]), "plaquette_spatial": float(P[1]),
                        "plaquette_temporal": float(P[2]), "polyakov": float(poly)},
    }
    rec["observables"]["kp_attempts_per_update"] = (c_end[0] - c_start[0]) / updates
    rec["observables"]["kp_cap_failures_per_update"] = (c_end[1] - c_start[1]) / updates
    if not args.no_extras:
        rec["host_transfer"] = host_transfer(su2, V, updates, ms_per_step * args.steps)
    su2.su2_finalize()
    check = None
    if not args.no_extras:
        for name in args.extra or EXTRAS:
            t_x = time.perf_counter()
            print(f"extra workload {name} ...", file=sys.stderr, flush=True)
            if name == "learned_proposal":
                rec[name] = learned_proposal(su2, sweeps=args.learned_sweeps)
            else:
                rec[name] = EXTRA_FUNCS[name](su2)
            print(f"extra workload {name} done in {time.perf_counter() - t_x:.1f} s", file=sys.stderr, flush=True)
        if "batched_replicas" in rec:
            check = rec["batched_replicas"].pop("_check")
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(w)
        if check is not None:
            rec["cpu_baseline"]["batched_replicas_vs_oracle"] = replica_check(*check)
    su2.su2_finalize()
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
