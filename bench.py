"""Benchmark of the MPMC hard-disk sampler on one MI355X.

Workload: N = 1024^2 disks at eta = 0.716 (the paper-scale system, Sec. IV),
triangular start, one trial per non-empty active cell, step tuned during
warm-up to about 30 % acceptance and then frozen.  One benchmark step is one
pass of the whole plain hot path over the box: `--sweeps` MPMC sweeps (random
grid shift + re-bin + four colour sub-sweeps each, replayed from a captured
HIP graph), then one contact-histogram accumulation (pressure, Sec. II.C.1)
and one psi_6 field evaluation (Eq. (8)), as logged every 100 sweeps.

Prints one JSON line: whole-job trial moves per second with the state resident
in HBM, the sweep kernel's roofline figures measured with HIP events on the
stream it runs on, and the CPU oracle timed on a bounded sample.
"""
import argparse
import json
import math
import os
import platform
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E, GB/s
# 32-bit vector ALU: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz, one operation per
# lane and clock (packed fp32 excluded), in tera-operations per second
ALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
N_DISKS = 1024 * 1024
ETA = 0.716
# Algorithmic 32-bit operations of one trial: one Philox4x32-10 block (10
# rounds of two 32x32->64 multiplies, counted as two operations each, and
# four xors: 80), slot pick and step (7), new position (2), in-cell test (4),
# accept (2): 95; plus one pair test (2 subtractions, 2 multiplications, 1
# addition, 1 comparison: 6) per other disk of the 3 x 3 cell neighbourhood.
# Philox's key schedule (nine additions of the Weyl constants per block) is not
# counted: the key is the seed, the same in every lane, so the round keys are
# scalar values that no vector lane computes.
ALU_OPS_TRIAL = 95
ALU_OPS_PAIR = 6


def algorithmic_bytes_per_sweep(N, M):
    """What one sweep must move at least: every position read and written
    (2 x 8 B per disk), every tag read and written (2 x 4 B per disk), every
    cell count read and written (2 x 1 B per cell)."""
    return 16 * N + 8 * N + 2 * M * M


def alu_ops_per_trial(N, M):
    """Algorithmic operations per trial with the mean number of other disks
    in a 3 x 3 block of cells, 9 N / M^2 - 1."""
    return ALU_OPS_TRIAL + ALU_OPS_PAIR * (9.0 * N / (M * M) - 1.0)


def max_step(box):
    """The largest step m the box allows: cell width plus step below 4."""
    return min(255, int(math.ceil((4.0 - box.info()["w"]) * 256.0)) - 1)


def tune_step(box, target=0.30, rounds=6, block=100):
    """Equilibration-only step tuning: m <- round(m * acc / target)."""
    m = box.info()["step_m"]
    acc = None
    for _ in range(rounds):
        t, a = box.sweep(block, counts=True)
        acc = a / t
        new = max(1, min(max_step(box), int(round(m * acc / target))))
        if new == m:
            break
        m = new
        box.set_step(m)
    return m, acc


def kernel_source_digest():
    """Digest of the sources that define the timed sweep kernel's code (its
    file and the common header of views, random numbers and constants; the
    launcher declarations of the other kernels are left out), to tell whether
    a stored counter profile still describes it."""
    import hashlib
    h = hashlib.sha256()
    for f in ("sweep_fused.hip", "mpmc_common.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1211_1645_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def stored_traffic():
    """HBM bytes per sweep launch from the committed rocprofv3 --pmc summary
    (FETCH_SIZE + WRITE_SIZE, scaled by the copy-kernel calibration), or None
    if it was taken on a different kernel source."""
    path = os.path.join(ROOT, "profiles", "traffic_k_fused_1024sq_eta0716.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    if d.get("kernel_digest") != kernel_source_digest():
        return None
    return d.get("bytes_per_launch")


def stored_tau():
    """The Psi_6 correlation time measured by `--workload tau` at the paper's
    speed-comparison point (N = 512^2, eta = 0.698), from its committed
    summary, or None."""
    path = os.path.join(ROOT, "profiles", "psi6_tau_512sq_eta0698.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    keys = ("tau_efold_displacements_per_disk", "tau_displacements_per_disk",
            "paper_tau_displacements_per_disk", "decorrelations_per_s", "sweeps_per_s",
            "tau_efold_mean_displacements_per_disk", "tau_efold_se_displacements_per_disk",
            "command")
    out = {k: d.get(k) for k in keys}
    out["independent_runs"] = len(d.get("independent_runs", [])) or 1
    out["N"], out["eta"], out["source"] = 512 * 512, 0.698, "profiles/psi6_tau_512sq_eta0698.json"
    out["provenance"] = ("stored: measured by the command above on an MI355X earlier, "
                         "read from profiles/psi6_tau_512sq_eta0698.json; not measured in this run")
    return out


def stored_tau_bound():
    """The Psi_6 correlation run at the benchmark's own point (N = 1024^2,
    eta = 0.716), from its committed summary, or None: a lower bound on tau,
    since the ordered box keeps its orientation through the run."""
    path = os.path.join(ROOT, "profiles", "psi6_tau_1024sq_eta0716.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    out = {k: d.get(k) for k in ("tau_sweeps_lower_bound", "decorrelations_per_s_upper_bound",
                                 "abs_Psi6_mean_after_discard", "orientation_drift_deg",
                                 "command")}
    out["source"] = "profiles/psi6_tau_1024sq_eta0716.json"
    out["provenance"] = ("stored: measured by the command above on an MI355X earlier, "
                         "read from profiles/psi6_tau_1024sq_eta0716.json; not measured in this run")
    return out


def stored_pressure():
    """The pressure measured by `--workload pressure` at the paper's test
    point (N = 256^2, eta = 0.698, Table I), from its committed summary, or
    None."""
    path = os.path.join(ROOT, "profiles", "pressure_256sq_eta0698.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    out = {k: d.get(k) for k in ("p_star", "se", "paper_p_star", "paper_se", "z_vs_paper",
                                 "displacements_per_run", "command")}
    out["N"], out["eta"], out["replicas"] = 256 * 256, 0.698, d["config"]["replicas"]
    out["source"] = "profiles/pressure_256sq_eta0698.json"
    out["provenance"] = ("stored: measured by the command above on an MI355X earlier, "
                         "read from profiles/pressure_256sq_eta0698.json; not measured in this run")
    return out


def copy_calibration(nbytes=512 << 20, reps=3):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    a = torch.empty(nbytes // 4, dtype=torch.float32, device="cuda")
    b = torch.empty_like(a)
    a.fill_(1.0)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_calibration_bytes": nbytes, "reps": reps}))


LEARN_STEP_FACTOR = 3


TC_SIDE, TC_ETA = 128, 0.66          # Psi_6 decorrelation comparison box


def train_learner(side, eta, seed, step_factor=LEARN_STEP_FACTOR):
    """A learned proposal for the box N = side^2 at eta on the w >= 3 grid:
    accepted plain moves at step_factor times the tuned step (so that the
    network learns the larger moves a neighbourhood allows), 3000 Adam
    steps of 8192.  Returns (learner, facts)."""
    import torch
    import paper_1211_1645_amd.mpmc as mp
    tb = mp.Box(side * side, eta, seed=seed + 1, step_m=40, cell_min=3.0, schedule="simple")
    m_train, _ = tune_step(tb)
    tb.sweep(2000)
    m_collect = min(max_step(tb), step_factor * m_train)
    tb.set_step(m_collect)
    L = mp.Learner(seed=seed + 2, capacity=1 << 22)
    n = 0
    while n < (1 << 21):
        n = L.collect(tb, 100)
    t0 = time.perf_counter()
    loss0 = L.train(1, batch=8192, lr=2e-3)
    loss = L.train(3000, batch=8192, lr=1e-3)
    torch.cuda.synchronize()
    return L, {"moves": n, "step_m": m_collect, "tuned_step_m": m_train,
               "adam_steps": 3001, "batch": 8192, "loss_first": loss0, "loss_last": loss,
               "seconds": time.perf_counter() - t0}


def psi6_runs(make_box, advance, runs, equil, sweeps, every, label):
    """`runs` independent boxes, one after the other, each with the GPU to
    itself: `equil` sweeps, then `sweeps` more with Psi_6 every `every`.
    Returns (series per run, elapsed seconds of the measured parts, trials
    per disk and sweep).  The runs are not overlapped on several streams:
    on this GPU kernels of at most two streams ran concurrently, so three
    boxes side by side took twice as long as one, whatever the sampler."""
    import numpy as np
    import torch
    n = sweeps // every
    series = np.zeros((runs, n), np.complex128)
    elapsed, trials = 0.0, 0
    stream = torch.cuda.Stream()
    for r in range(runs):
        with torch.cuda.stream(stream):
            b = make_box(r, stream.cuda_stream)
        advance(b, equil)
        torch.cuda.synchronize()
        i0 = b.info()
        t0 = time.perf_counter()
        last = t0
        for k in range(n):
            advance(b, every)
            series[r, k] = b.psi6()
            if time.perf_counter() - last > 30:
                last = time.perf_counter()
                progress("%s run %d: %d of %d sweeps" % (label, r, (k + 1) * every, sweeps))
        torch.cuda.synchronize()
        elapsed += time.perf_counter() - t0
        trials += b.info()["trials"] - i0["trials"]
        N = b.N
        del b
    disp = trials / (runs * n * every * N)
    return series, elapsed, disp


def efold(series, maxlag):
    """First lag at which C(dt) of Eq. (9) falls below 1/e (NaN if never)."""
    import numpy as np
    import paper_1211_1645_amd.mpmc as mp
    Cv = mp.acf(series, maxlag)
    below = np.nonzero(Cv < math.exp(-1.0))[0]
    return float(below[0]) if len(below) else float("nan")


def phases_bench(args):
    """Per-phase profile of the sweep kernel on the benchmark's box: device
    clock stamps at the phase boundaries of every tile (mpmc_profile_phases),
    mean microseconds per tile."""
    import paper_1211_1645_amd.mpmc as mp
    box = mp.Box(N_DISKS, ETA, seed=args.seed, step_m=20, lattice="triangular",
                 schedule="fused" if args.tile else "auto", tile=args.tile)
    step_m, _ = tune_step(box)
    box.sweep(200)
    info = box.info()
    ph = box.profile_phases(50)
    print(json.dumps({"workload": "phase profile of the sweep kernel, N=1024^2 eta=0.716, "
                                  "step m=%d, tile %d, 50 sweeps" % (step_m, info["tile"]),
                      "tile": info["tile"], "us_per_tile": ph,
                      "share": {k: ph[k] / ph["tile"] for k in ("load", "pass1", "pass2", "pass3",
                                                                 "pass4", "rebin_classes",
                                                                 "rebin_scatter")},
                      "kernel_digest": kernel_source_digest()}))


def tau_compare_bench(args):
    """Psi_6 decorrelation of the learned proposal against the plain one
    (Sec. III, Eq. (9); Table II's units): N = side^2 at eta, three
    independent runs per sampler, each about 100 plain correlation times
    long after equilibration.  Samplers: plain on the w >= 3 grid (the
    learned proposal's grid), plain on its own w >= 2 grid (the fused
    kernel), learned on the w >= 3 grid.  tau is the e-folding lag of
    C(dt); the rate is sweeps per second, each run alone on the GPU, divided
    by tau in sweeps."""
    import numpy as np
    import paper_1211_1645_amd.mpmc as mp
    side, eta, R = args.tc_side, args.tc_eta, 3
    L, train = train_learner(side, eta, args.seed)
    progress("tau-compare: learned proposal trained (%d moves)" % train["moves"])
    probe = mp.Box(side * side, eta, seed=args.seed, step_m=40, cell_min=3.0, schedule="simple")
    m3, _ = tune_step(probe)
    probe2 = mp.Box(side * side, eta, seed=args.seed, step_m=40)
    m2, _ = tune_step(probe2)
    every, sweeps, equil = args.tc_every, args.tc_sweeps, args.tc_equil
    samplers = {
        "plain_w3": (lambda r, st: mp.Box(side * side, eta, seed=args.seed + 10 + r, step_m=m3,
                                          cell_min=3.0, schedule="simple", stream=st),
                     lambda b, k: b.sweep(k)),
        "plain_w2_fused": (lambda r, st: mp.Box(side * side, eta, seed=args.seed + 20 + r,
                                                step_m=m2, stream=st),
                           lambda b, k: b.sweep(k)),
        "learned_w3": (lambda r, st: mp.Box(side * side, eta, seed=args.seed + 30 + r, step_m=m3,
                                            cell_min=3.0, schedule="simple", stream=st),
                       None),
    }
    out = {}
    for name, (make, adv) in samplers.items():
        if adv is None:
            # equilibrated by the plain sweep, then measured with the learned
            # proposal
            def make_eq(r, st, make=make):
                b = make(r, st)
                b.sweep(equil)
                return b
            series, el, disp = psi6_runs(make_eq, lambda b, k: mp.sweep_learned(b, L, k, eps=args.tc_eps),
                                         R, 0, sweeps, every, name)
        else:
            series, el, disp = psi6_runs(make, adv, R, equil, sweeps, every, name)
        taus = np.array([efold(x, len(x) // 4) * every for x in series])
        rate = R * sweeps / el
        tm, tse = float(np.mean(taus)), float(np.std(taus, ddof=1) / math.sqrt(R))
        out[name] = {"tau_sweeps_runs": taus.tolist(), "tau_sweeps": tm, "tau_sweeps_se": tse,
                     "tau_trials_per_disk": tm * disp, "tau_trials_per_disk_se": tse * disp,
                     "trials_per_disk_per_sweep": disp, "sweeps_per_s": rate,
                     "us_per_sweep": 1e6 / rate,
                     "decorrelations_per_s": rate / tm,
                     "decorrelations_per_s_se": rate / tm * tse / tm,
                     "abs_Psi6_mean": float(np.abs(series).mean()),
                     "run_length_in_tau": sweeps / tm}
        progress("tau-compare: %s tau = %.0f +- %.0f sweeps, %.3g decorrelations/s" %
                 (name, tm, tse, rate / tm))
    base = out["plain_w3"]
    lr = out["learned_w3"]
    line = {
        "metric": "psi6-decorrelations/s, learned against plain, %d^2 disks eta=%.2f" % (side, eta),
        "value": lr["decorrelations_per_s"], "unit": "decorrelations/s",
        "n_gpus": 1, "steps": sweeps // every, "warmup": equil,
        "ms_per_step": None, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f32 (sampler), f64 (proposal law)",
        "data": "synthetic (triangular-lattice starts, Philox4x32-10 seeds %d..)" % args.seed,
        "config": {"workload": "Psi6 decorrelation, N=%d^2 eta=%.2f, %d runs per sampler one "
                               "after the other, %d sweeps each after %d, Psi6 every %d; learned "
                               "eps=%.2f"
                               % (side, eta, R, sweeps, equil, every, args.tc_eps),
                   "N": side * side, "eta": eta, "step_m_w3": m3, "step_m_w2": m2},
        "train": train,
        "samplers": out,
        "gain_tau_per_sweep_vs_plain_w3": base["tau_sweeps"] / lr["tau_sweeps"],
        "gain_tau_per_trial_vs_plain_w3": base["tau_trials_per_disk"] / lr["tau_trials_per_disk"],
        "gain_decorrelations_per_s_vs_plain_w3": lr["decorrelations_per_s"] /
                                                  base["decorrelations_per_s"],
        "gain_decorrelations_per_s_vs_plain_w2_fused": lr["decorrelations_per_s"] /
                                                        out["plain_w2_fused"]["decorrelations_per_s"],
        "command": "python3 bench.py --workload tau-compare --tc-side %d --tc-eta %.2f --tc-sweeps %d "
                   "--tc-equil %d --tc-every %d --tc-eps %.2f" % (side, eta, sweeps, equil, every,
                                                               args.tc_eps),
    }
    print(json.dumps(line))


def stored_tau_compare():
    """The learned-against-plain decorrelation comparison from its committed
    summary (`--workload tau-compare`), or None."""
    path = os.path.join(ROOT, "profiles", "psi6_tau_learned_vs_plain_128sq_eta066.json")
    if not os.path.exists(path):
        return None
    d = json.load(open(path))
    out = {k: d.get(k) for k in ("gain_tau_per_sweep_vs_plain_w3", "gain_tau_per_trial_vs_plain_w3",
                                 "gain_decorrelations_per_s_vs_plain_w3",
                                 "gain_decorrelations_per_s_vs_plain_w2_fused", "command")}
    out["decorrelations_per_s"] = {k: [v["decorrelations_per_s"], v["decorrelations_per_s_se"]]
                                   for k, v in d["samplers"].items()}
    out["tau_sweeps"] = {k: [v["tau_sweeps"], v["tau_sweeps_se"]] for k, v in d["samplers"].items()}
    out["provenance"] = ("stored: measured by the command above on an MI355X earlier, read from "
                         "profiles/psi6_tau_learned_vs_plain_128sq_eta066.json; not measured in "
                         "this run")
    return out


def learned_speed(seed):
    """Sweep cost of the learned proposal against the plain one, live: at the
    decorrelation-comparison box and at N = 1024^2 (w >= 3 grid, simple
    schedule for plain), microseconds per sweep."""
    import torch
    import paper_1211_1645_amd.mpmc as mp
    L = mp.Learner(seed=seed + 2, capacity=16)
    out = {}
    for side in (TC_SIDE, 1024):
        b = mp.Box(side * side, TC_ETA if side == TC_SIDE else ETA, seed=seed + 3, step_m=40,
                   cell_min=3.0, schedule="simple")
        res = {}
        for mode, run in (("plain_w3", lambda k: b.sweep(k)),
                          ("learned_w3", lambda k: mp.sweep_learned(b, L, k, eps=0.1))):
            run(4)
            torch.cuda.synchronize()
            t = time.perf_counter()
            run(40)
            torch.cuda.synchronize()
            res[mode + "_sweep_us"] = (time.perf_counter() - t) / 40 * 1e6
        out["N=%d^2" % side] = res
    return out


# Algorithmic operations of one structure-factor term (one disk, one wave
# vector) as k_rho evaluates it (fp64 vector arithmetic issues at the 32-bit
# rate on this chip: 78.6 TFLOP/s of fp64 FMA = 256 CUs x 64 lanes x 2.4 GHz
# x 2): the scaled phase h x + k y (2 fp64), its integer part and fraction
# (2), conversion and scaling of the fraction (2), the table index (2), the
# table read (1), the squared residual angle (1), its cosine and sine from the
# Taylor series (5), the rotation by the table entry (4) and the two fp64
# accumulations with their conversions (4): 23.
ALU_OPS_RHO_TERM = 23.0


def positional_bench(args):
    """Positional order (Sec. IV.C, IV.D) on an equilibrating N = 1024^2 box at
    eta = 0.716: the structure-factor scan for q0, chi_j, and C_q0(r) out to
    r = 100 sigma."""
    import math
    import numpy as np
    import torch
    import paper_1211_1645_amd.mpmc as mp
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        box = mp.Box(N_DISKS, ETA, seed=args.seed, step_m=20, lattice="triangular",
                     stream=stream.cuda_stream)
        box.sweep(200)
        info = box.info()
        L = info["L_eff"]
        a0 = math.sqrt(2.0 / (math.sqrt(3.0) * info["N"] / L ** 2))
        qp = 4 * math.pi / (math.sqrt(3.0) * a0)
        unit = 2 * math.pi / L
        # one launch worth of wave vectors (65536) in the annulus sector
        r = int(math.ceil(1.1 * qp / unit))
        k, h = np.meshgrid(np.arange(-r, r + 1), np.arange(-r, r + 1), indexing="ij")
        h, k = h.ravel(), k.ravel()
        n = np.hypot(h, k) * unit
        ang = np.arctan2(k, h)
        sel = (n >= 0.9 * qp) & (n <= 1.1 * qp) & (ang >= 0) & (ang < math.pi / 3)
        hk = np.stack([h[sel], k[sel]], 1)[:65536].astype(np.int32)
        box.structure_factor(hk[:256])   # warm-up
        times = []
        for _ in range(args.steps):
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record(stream)
            S = box.structure_factor(hk)
            e1.record(stream)
            torch.cuda.synchronize()
            times.append(e0.elapsed_time(e1) * 1e-3)
        t_s = sum(times) / len(times)
        terms = float(len(hk)) * info["N"]
        t0 = time.perf_counter()
        hq, kq, Sq = box.find_q0(0.9 * qp, 1.1 * qp, 0.0, math.pi / 3)
        torch.cuda.synchronize()
        t_find = time.perf_counter() - t0
        t0 = time.perf_counter()
        chi, field = box.chi_field(hq, kq)
        torch.cuda.synchronize()
        t_chi = time.perf_counter() - t0
        qx, qy = unit * hq, unit * kq
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        num, cnt = box.cq(qx, qy, 1.0, 100)
        e1.record(stream)
        torch.cuda.synchronize()
        t_cq = e0.elapsed_time(e1) * 1e-3
    achieved = terms * ALU_OPS_RHO_TERM / t_s / 1e12
    line = {
        "metric": "structure-factor terms/s (disk x wave vector), 1024^2 disks eta=0.716",
        "value": terms / t_s,
        "unit": "terms/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": 1,
        "ms_per_step": t_s * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64 phase, f32 rotation, f64 sums",
        "data": "synthetic (triangular start, 200 sweeps, Philox4x32-10 seed %d)" % args.seed,
        "config": {"workload": "positional order: S(q) at %d allowed wave vectors of the "
                               "annulus sector 0.9-1.1 x 4pi/(sqrt3 a0), 0-60 deg; q0 search "
                               "over the whole sector; chi_j; C_q0(r) for r = 0..99 sigma"
                               % len(hk), "N": info["N"], "eta": ETA, "M": info["M"]},
        "q0": {"h": hq, "k": kq, "S": Sq, "q": math.hypot(qx, qy), "search_s": t_find},
        "chi_s": t_chi,
        "cq": {"seconds": t_cq, "bins": 100, "dr": 1.0, "pairs": int(cnt.sum()),
               "C_at_10_50_99": [float(num[i] / cnt[i]) for i in (10, 50, 99)]},
        "roofline": {"bound": "alu", "achieved": achieved, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved / ALU_PEAK_TOPS, "traffic": None,
                     "kernel": "k_rho (one launch of %d wave vectors)" % len(hk),
                     "ops_per_term": ALU_OPS_RHO_TERM},
    }
    if not args.no_cpu_baseline:
        from oracle.orc import OracleBox
        o = OracleBox(N_DISKS, ETA, seed=args.seed, lattice=1, step_m=20)
        o.sweep(1)
        t0 = time.perf_counter()
        o.structure_factor(hk[:8])
        one = (time.perf_counter() - t0) / 8
        nq = max(8, min(len(hk), int(15.0 / max(one, 1e-6))))
        t0 = time.perf_counter()
        o.structure_factor(hk[:nq])
        dt = time.perf_counter() - t0
        line["cpu_baseline"] = dict(
            value=nq * float(info["N"]) / dt, unit="terms/s", cores=1, kind="oracle",
            sample="S(q) at %d of the same wave vectors on the oracle's N=1024^2 box after one "
                   "sweep (%.1f s, 1 thread of %s)" % (nq, dt, host_cpu()))
    print(json.dumps(line))


TAU_ETA = 0.698
TAU_PAPER_DISP = 8.0e5   # MPMC correlation time of Psi_6 in displacements per disk (Table II)


def batch_bench(args):
    """Many independent boxes of uneven size and density swept together: 64
    boxes with N drawn from {64^2, 96^2, 128^2, 192^2, 256^2} and eta uniform
    in [0.69, 0.73] (seeded), one persistent graph-captured launch per sweep,
    against the same boxes each swept by its own launches (fused kernel,
    autotuned shape, graphs)."""
    import numpy as np
    import torch
    import paper_1211_1645_amd.mpmc as mp
    from paper_1211_1645_amd.workloads import batch_boxes
    N, eta, seeds = batch_boxes(64, seed=args.seed)
    b = mp.Batch(N, eta, seeds, step_m=40)
    b.set_graphs(args.sweeps)
    b.sweep(args.sweeps)
    torch.cuda.synchronize()
    inf = b.info()
    k = args.steps * args.sweeps
    t0 = time.perf_counter()
    tr, ac = b.sweep(k, counts=True)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    for _ in range(2):
        b.accumulate_contacts()
        b.sweep(10)
    progress("batch: %d sweeps of %d boxes in %.3f s" % (k, len(N), dt))
    # the same boxes one at a time
    boxes = [mp.Box(int(n), float(e), seed=int(sd), step_m=40) for n, e, sd in zip(N, eta, seeds)]
    for bx in boxes:
        bx.set_graphs(args.sweeps)
        bx.sweep(args.sweeps)
    torch.cuda.synchronize()
    ks = max(args.sweeps, k // 4)
    t0 = time.perf_counter()
    tr1 = 0
    for bx in boxes:
        i0 = bx.info()["trials"]
        bx.sweep(ks)
        torch.cuda.synchronize()
        tr1 += bx.info()["trials"] - i0
    dt1 = time.perf_counter() - t0
    line = {
        "metric": "trial moves/s, 64-box batch (N from 64^2 to 256^2, eta 0.69-0.73)",
        "value": tr / dt, "unit": "trial moves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": 1,
        "ms_per_step": dt / args.steps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (triangular-lattice starts, Philox4x32-10 seeds %d..%d)" %
                (args.seed, args.seed + 63),
        "config": {"workload": "64 independent boxes, one persistent launch per sweep, %d "
                               "sweeps per step" % args.sweeps,
                   "N_total": int(N.sum()), "tile": inf["tile"], "threads": inf["threads"]},
        "batch_sweep_us": dt / k * 1e6,
        "acceptance": ac / max(tr, 1),
        "one_box_at_a_time": {"trial_moves_per_s": tr1 / dt1,
                              "sweep_of_all_boxes_us": dt1 / ks * 1e6},
        "speedup_over_one_at_a_time": (tr / dt) / (tr1 / dt1),
        "P_star_first_boxes": [float(x) for x in b.measure_pressure()[0][:4]],
    }
    print(json.dumps(line))


SCALE_N = 4096 * 4096


def scale_bench(args):
    """The plain sweep on the scale probe N = 4096^2 (16.8 M disks, state
    of about 440 MB per sweep, beyond the 256 MB Infinity Cache): sweeps/s,
    trial moves/s and the roofline fractions of the same kernel."""
    import torch
    import paper_1211_1645_amd.mpmc as mp
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        box = mp.Box(SCALE_N, ETA, seed=args.seed, step_m=55, lattice="triangular",
                     schedule="fused" if args.tile else "auto", tile=args.tile,
                     stream=stream.cuda_stream)
        box.set_graphs(args.sweeps)
        step_m, _ = tune_step(box, block=20)
        info = box.info()
        progress("scale probe: M=%d schedule %d tile %d m=%d" %
                 (info["M"], info["schedule"], info["tile"], step_m))
        for _ in range(args.warmup):
            box.sweep(args.sweeps)
        torch.cuda.synchronize()
        t_before = box.info()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(args.steps):
            box.sweep(args.sweeps)
        e1.record(stream)
        torch.cuda.synchronize()
        t_after = box.info()
        overlaps, bad = box.validate()
    k = args.steps * args.sweeps
    sweep_s = e0.elapsed_time(e1) * 1e-3 / k
    trials = t_after["trials"] - t_before["trials"]
    bytes_per = algorithmic_bytes_per_sweep(info["N"], info["M"])
    ops_per = trials / k * alu_ops_per_trial(info["N"], info["M"])
    line = {
        "metric": "trial moves/s, 4096^2 disks eta=0.716 (scale probe)",
        "value": trials / (sweep_s * k), "unit": "trial moves/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": sweep_s * args.sweeps * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (triangular-lattice start, Philox4x32-10 seed %d)" % args.seed,
        "config": {"workload": "plain MPMC scale probe, N=4096^2, eta=0.716, step tuned to "
                               "~30%% acceptance (m=%d), %d sweeps per step" % (step_m, args.sweeps),
                   "N": info["N"], "M": info["M"], "tile": info["tile"],
                   "schedule": "fused" if info["schedule"] == 2 else "simple"},
        "sweep_us": sweep_s * 1e6,
        "acceptance": (t_after["accepts"] - t_before["accepts"]) / max(trials, 1),
        "validate": {"overlaps": overlaps, "bad": bad},
        "roofline": {"bound": "alu", "achieved": ops_per / sweep_s / 1e12, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": ops_per / sweep_s / 1e12 / ALU_PEAK_TOPS,
                     "traffic": None, "kernel": "k_fused (one sweep per launch)",
                     "hbm": {"achieved": bytes_per / sweep_s / 1e9, "peak": HBM_PEAK_GBS,
                             "unit": "GB/s", "frac": bytes_per / sweep_s / 1e9 / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_launch": bytes_per}},
    }
    print(json.dumps(line))


def tau_analysis(series, sample, disp_per_sweep, discard):
    """tau of a Psi_6 series sampled every `sample` sweeps: the exponential
    fit of Sec. III over 0.05 <= C <= 0.5, the e-folding lag (first C < 1/e,
    the larger and so the conservative figure for runs of a few tens of tau,
    which the decorrelation rate uses) and the integrated time, for the whole
    series after
    `discard` sweeps and for its two halves, in displacements per disk."""
    import math
    import numpy as np
    import paper_1211_1645_amd.mpmc as mp
    x = np.asarray(series)[discard // sample:]
    unit = sample * disp_per_sweep

    def one(part):
        Cv = mp.acf(part, len(part) // 4)
        try:
            t, ti = mp.tau(Cv, 0.05, 0.5)
        except mp.MPMCError:   # too short for the exponential tail
            t, ti = float("nan"), float("nan")
        below = np.nonzero(Cv < math.exp(-1.0))[0]
        ef = float(below[0]) if len(below) else float("nan")
        return t * unit, ef * unit, ti * unit

    t, ef, ti = one(x)
    halves = [one(x[:len(x) // 2]), one(x[len(x) // 2:])]
    return {"tau_sweeps": t * sample / unit, "tau_displacements_per_disk": t,
            "tau_efold_displacements_per_disk": ef, "tau_int_displacements_per_disk": ti,
            "tau_halves_displacements_per_disk": [h[0] for h in halves],
            "tau_efold_halves_displacements_per_disk": [h[1] for h in halves],
            "run_length_in_tau": len(x) * unit / t if t == t else None,
            "abs_Psi6_mean": float(np.abs(x).mean())}


def tau_bench(args):
    """Psi_6 correlation time of the plain sampler, by default at the
    configuration of the paper's speed comparison (N = 512^2, eta = 0.698,
    Table II; --tau-side and --tau-eta choose another box): a long run
    from the triangular start, Psi_6 every `sample` sweeps (one graph replay
    each), the first `discard` sweeps dropped, C(dt) of Eq. (9) over all time
    origins, tau from the exponential tail (Sec. III)."""
    import numpy as np
    import torch
    import paper_1211_1645_amd.mpmc as mp
    sample = args.tau_sample
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        box = mp.Box(args.tau_side ** 2, args.tau_eta, seed=args.seed, step_m=20,
                     lattice="triangular", stream=stream.cuda_stream)
        box.set_graphs(sample)
        step_m, acc = tune_step(box)
        info = box.info()
        progress("tau run: N=%d eta=%.3f m=%d schedule %d tile %d" %
                 (info["N"], args.tau_eta, step_m, info["schedule"], info["tile"]))
        n_samples = args.tau_sweeps // sample
        series = np.zeros(n_samples, np.complex128)
        i0 = box.info()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        last = t0
        for k in range(n_samples):
            box.sweep(sample)
            series[k] = box.psi6()
            now = time.perf_counter()
            if now - last > 30.0:
                progress("tau run: %d of %d sweeps, |Psi6| = %.3f" %
                         ((k + 1) * sample, n_samples * sample, abs(series[k])))
                if args.tau_series:  # the series so far, in case the run is cut short
                    np.save(args.tau_series, series[:k + 1])
                last = now
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        i1 = box.info()
    if args.tau_series:
        np.save(args.tau_series, series)
    disp_per_sweep = (i1["trials"] - i0["trials"]) / (n_samples * sample) / info["N"]
    res = tau_analysis(series, sample, disp_per_sweep, args.tau_discard)
    sweeps_per_s = n_samples * sample / elapsed
    paper_point = (args.tau_side, args.tau_eta) == (512, TAU_ETA)
    where = ("plain MPMC at the paper's speed-comparison point, N=512^2, eta=0.698"
             if paper_point else "plain MPMC, N=%d^2, eta=%.3f" % (args.tau_side, args.tau_eta))
    line = {
        "metric": "psi6-decorrelation sweeps/s (sweeps/s / tau), %d^2 disks eta=%.3f" %
                  (args.tau_side, args.tau_eta),
        "value": sweeps_per_s * disp_per_sweep / res["tau_efold_displacements_per_disk"],
        "unit": "decorrelations/s",
        "n_gpus": 1, "steps": n_samples, "warmup": 0,
        "ms_per_step": elapsed / n_samples * 1e3,
        "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (triangular start, Philox4x32-10 seed %d)" % args.seed,
        "config": {"workload": "%s, step tuned to ~30%% acceptance (m=%d); %d sweeps, "
                               "Psi6 every %d, first %d discarded" %
                               (where, step_m, n_samples * sample, sample, args.tau_discard),
                   "N": info["N"], "eta": args.tau_eta, "M": info["M"], "tile": info["tile"]},
        "sweeps_per_s": sweeps_per_s,
        "trial_moves_per_s": (i1["trials"] - i0["trials"]) / elapsed,
        "displacements_per_disk_per_sweep": disp_per_sweep,
        "tau_sweeps": res["tau_sweeps"],
        "paper_tau_displacements_per_disk": TAU_PAPER_DISP if paper_point else None,
    }
    line.update(res)
    print(json.dumps(line))


PRESSURE_N, PRESSURE_ETA = 256 * 256, 0.698
PRESSURE_PAPER = (9.17078, 4.5e-5)   # MPMC pressure and standard error (Table I)


def batch_pressure_blocks(b, n_blocks, block, sample, label):
    """P* of every box of batch `b` for each of `n_blocks` blocks of `block`
    sweeps, the contact histogram accumulated every `sample` sweeps and reset
    at the start of each block: (P[block, box], trial moves, seconds)."""
    import numpy as np
    import torch
    boxes = [b.box(i) for i in range(b.n)]
    per_block = block // sample
    P = np.zeros((n_blocks, b.n))
    trials = 0
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    last = t0
    for blk in range(n_blocks):
        for bx in boxes:
            bx.reset_contacts()
        for _ in range(per_block):
            t, _a = b.sweep(sample, counts=True)
            trials += t
            b.accumulate_contacts()
        P[blk] = b.measure_pressure()[0]
        now = time.perf_counter()
        if now - last > 20.0 or blk == n_blocks - 1:
            progress("%s: %d of %d sweeps, block mean P* = %.5f" %
                     (label, (blk + 1) * block, n_blocks * block, P[blk].mean()))
            last = now
    torch.cuda.synchronize()
    return P, trials, time.perf_counter() - t0


def pressure_bench(args):
    """The pressure at the paper's test point (N = 256^2, eta = 0.698, Table
    I): independent replicas from triangular starts (Philox keys seed + 100 +
    r) swept together as one batch, the contact histogram accumulated every
    `p_sample` sweeps and fitted per replica and block of `p_block` sweeps;
    blocks that end within the first `p_equil` sweeps are dropped.  The
    standard error comes from the scatter of the replica means."""
    import numpy as np
    import torch
    import paper_1211_1645_amd.mpmc as mp
    R = args.p_replicas
    tb = mp.Box(PRESSURE_N, PRESSURE_ETA, seed=args.seed + 99, step_m=20)
    step_m, _ = tune_step(tb)
    tb.close()
    seeds = np.arange(args.seed + 100, args.seed + 100 + R, dtype=np.uint64)
    b = mp.Batch(np.full(R, PRESSURE_N, np.uint32), np.full(R, PRESSURE_ETA), seeds, step_m=step_m)
    b.set_graphs(args.p_sample)
    inf = b.info()
    progress("pressure run: %d replicas of N=%d, eta=%.3f, m=%d, tile %d" %
             (R, PRESSURE_N, PRESSURE_ETA, step_m, inf["tile"]))
    n_blocks = (args.p_equil + args.p_sweeps) // args.p_block
    P, trials, elapsed = batch_pressure_blocks(b, n_blocks, args.p_block, args.p_sample,
                                               "pressure run")
    keep = P[args.p_equil // args.p_block:]
    rep = keep.mean(axis=0)
    mean = float(rep.mean())
    se = float(rep.std(ddof=1) / math.sqrt(R))
    paper, paper_se = PRESSURE_PAPER
    sweeps = n_blocks * args.p_block
    line = {
        "metric": "P* = beta P (2 sigma)^2 at N=256^2, eta=0.698 (Table I)",
        "value": mean, "unit": "dimensionless",
        "n_gpus": 1, "steps": n_blocks, "warmup": 0,
        "ms_per_step": elapsed / n_blocks * 1e3,
        "higher_is_better": None, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (triangular starts, Philox4x32-10 seeds %d..%d)" %
                (args.seed + 100, args.seed + 99 + R),
        "config": {"workload": "%d independent replicas of N=256^2 at eta=0.698 in one batch, "
                               "step tuned to ~30%% acceptance (m=%d); %d sweeps each, contact "
                               "histogram every %d sweeps, blocks of %d sweeps, first %d "
                               "sweeps discarded" %
                               (R, step_m, sweeps, args.p_sample, args.p_block, args.p_equil),
                   "N": PRESSURE_N, "eta": PRESSURE_ETA, "replicas": R,
                   "hist_bins": 100, "hist_dr_sigma": 1e-3, "fit_order": 4},
        "p_star": mean, "se": se,
        "paper_p_star": paper, "paper_se": paper_se,
        "z_vs_paper": (mean - paper) / math.sqrt(se * se + paper_se * paper_se),
        "replica_means": rep.tolist(),
        "block_means": P.mean(axis=1).tolist(),
        "displacements_per_run": trials / R,
        "trial_moves_per_s": trials / elapsed,
        "seconds": elapsed,
    }
    print(json.dumps(line))


EOS_ETAS = tuple(round(0.696 + 0.002 * i, 3) for i in range(15))   # 0.696 ... 0.724
EOS_SIZES = ((128 * 128, 3), (256 * 256, 2))                        # (N, replicas)


def eos_bench(args):
    """Equation of state across the coexistence region (Sec. IV.A): boxes of
    N = 128^2 and 256^2 at eta = 0.696 ... 0.724 (step 0.002), several
    replicas each, all swept together as one batch from triangular starts;
    P* per box and block as in the pressure workload, the first `p_equil`
    sweeps dropped; then the Mayer-Wood loop analysis of each size (cubic and
    quintic fits in v = pi / eta) and the exponent of beta Delta f(N)."""
    import numpy as np
    import paper_1211_1645_amd.mpmc as mp
    Ns, etas, seeds = [], [], []
    for N, R in EOS_SIZES:
        for e in EOS_ETAS:
            for r in range(R):
                Ns.append(N)
                etas.append(e)
                seeds.append(args.seed + 200 + len(seeds))
    tb = mp.Box(256 * 256, 0.710, seed=args.seed + 199, step_m=20)
    step_m, _ = tune_step(tb)
    tb.close()
    b = mp.Batch(np.asarray(Ns, np.uint32), np.asarray(etas), np.asarray(seeds, np.uint64),
                 step_m=step_m)
    b.set_graphs(args.p_sample)
    inf = b.info()
    progress("eos run: %d boxes, %d disks, m=%d, tile %d" % (b.n, sum(Ns), step_m, inf["tile"]))
    n_blocks = (args.p_equil + args.p_sweeps) // args.p_block
    P, trials, elapsed = batch_pressure_blocks(b, n_blocks, args.p_block, args.p_sample, "eos run")
    keep = P[args.p_equil // args.p_block:].mean(axis=0)
    Ns, etas = np.asarray(Ns), np.asarray(etas)
    sizes = []
    for N, R in EOS_SIZES:
        p, se = [], []
        for e in EOS_ETAS:
            v = keep[(Ns == N) & (etas == e)]
            p.append(float(v.mean()))
            se.append(float(v.std(ddof=1) / math.sqrt(len(v))))
        loops = {}
        for order in (3, 5):
            try:
                loops["order%d" % order] = mp.eos_loop(np.asarray(EOS_ETAS), np.asarray(p),
                                                       order=order)
            except mp.MPMCError as err:
                loops["order%d" % order] = {"error": str(err)}
        sizes.append({"N": int(N), "replicas": R, "eta": list(EOS_ETAS), "p_star": p, "se": se,
                      "loop": loops})
        progress("eos N=%d: %s" % (N, " ".join("%.4f" % x for x in p)))
    expo = {}
    for order in ("order3", "order5"):
        df = [sz["loop"][order].get("delta_f") for sz in sizes]
        if all(x is not None and x > 0 for x in df):
            expo[order] = mp.power_law(np.asarray([sz["N"] for sz in sizes], np.float64),
                                       np.asarray(df))[0]
    sweeps = n_blocks * args.p_block
    line = {
        "metric": "equation of state P*(eta) and Mayer-Wood loop, N=128^2 and 256^2",
        "value": trials / elapsed, "unit": "trial moves/s",
        "n_gpus": 1, "steps": n_blocks, "warmup": 0,
        "ms_per_step": elapsed / n_blocks * 1e3,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (triangular starts, Philox4x32-10 seeds %d..%d)" %
                (args.seed + 200, args.seed + 199 + b.n),
        "config": {"workload": "%d boxes (N=128^2 x3 and 256^2 x2 replicas at 15 densities "
                               "0.696-0.724) in one batch, m=%d; %d sweeps each, contact "
                               "histogram every %d sweeps, blocks of %d sweeps, first %d "
                               "discarded" % (b.n, step_m, sweeps, args.p_sample, args.p_block,
                                              args.p_equil),
                   "boxes": b.n, "disks": int(Ns.sum())},
        "sizes": sizes,
        "delta_f_exponent": expo,
        "paper_extrema_eta": [0.702, 0.714],
        "seconds": elapsed,
        "block_P": P.tolist(),
    }
    print(json.dumps(line))


def cpu_baseline(start_sweeps, seed, step_m, target_seconds=15.0):
    """The oracle (single thread) on the same start and step: sweeps of the
    full 1024^2 box until about target_seconds of CPU work."""
    from oracle.orc import OracleBox
    o = OracleBox(N_DISKS, ETA, seed=seed, lattice=1, step_m=step_m)
    t0 = time.perf_counter()
    o.sweep(1)
    one = time.perf_counter() - t0
    k = max(1, int(target_seconds / max(one, 1e-3)) - 1)
    i0 = o.info()
    t0 = time.perf_counter()
    o.sweep(k)
    dt = time.perf_counter() - t0
    i1 = o.info()
    return dict(value=(i1["trials"] - i0["trials"]) / dt, unit="trial moves/s", cores=1,
                kind="oracle",
                sample="%d sweeps of the N=1024^2 eta=0.716 box after 1 from the same "
                       "triangular start (%.1f s, 1 thread of %s)" % (k, dt, host_cpu()),
                build="gcc -O2 -ffp-contract=off -fno-fast-math")


def host_cpu():
    """CPU model and logical CPU count of the host, from /proc/cpuinfo."""
    model = platform.processor() or platform.machine()
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    return "%s, %d logical CPUs" % (model, os.cpu_count() or 0)


def progress(msg):
    print("bench: " + msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--sweeps", type=int, default=100, help="sweeps per benchmark step")
    ap.add_argument("--seed", type=int, default=0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-learned", action="store_true")
    ap.add_argument("--workload",
                    choices=("sweep", "positional", "tau", "scale", "batch", "pressure", "eos",
                             "tau-compare", "phases"),
                    default="sweep",
                    help="sweep: the sampler (default); positional: S(q), chi_j, C_q0(r); "
                         "tau: Psi6 correlation time at N=512^2, eta=0.698 (minutes); "
                         "scale: the sweep at N=4096^2; batch: 64 boxes in one launch; "
                         "pressure: P* at N=256^2, eta=0.698 over replicas (minutes); "
                         "eos: P*(eta) and its loop at N=128^2 and 256^2 (minutes); "
                         "tau-compare: Psi6 decorrelation, learned against plain (minutes); "
                         "phases: per-phase profile of the sweep kernel")
    ap.add_argument("--tau-side", type=int, default=512, help="tau run: N = side^2")
    ap.add_argument("--tau-eta", type=float, default=TAU_ETA)
    ap.add_argument("--tau-sweeps", type=int, default=20000000)
    ap.add_argument("--tau-discard", type=int, default=4000000)
    ap.add_argument("--tau-sample", type=int, default=1000)
    ap.add_argument("--tau-series", default="", help="save the Psi6 series (.npy)")
    ap.add_argument("--p-replicas", type=int, default=16)
    ap.add_argument("--p-equil", type=int, default=2000000)
    ap.add_argument("--p-sweeps", type=int, default=4000000)
    ap.add_argument("--p-block", type=int, default=250000)
    ap.add_argument("--p-sample", type=int, default=100)
    ap.add_argument("--tc-side", type=int, default=TC_SIDE)
    ap.add_argument("--tc-eta", type=float, default=TC_ETA)
    ap.add_argument("--tc-sweeps", type=int, default=240000)
    ap.add_argument("--tc-equil", type=int, default=20000)
    ap.add_argument("--tc-every", type=int, default=40)
    ap.add_argument("--tc-eps", type=float, default=0.1)
    ap.add_argument("--tile", type=int, default=0,
                    help="fix the fused sweep's tile (cells per side) instead of autotuning it; "
                         "for counter runs, whose serialised launches distort the autotuner")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of known size (for counter scaling)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the sampler runs one box per GPU and the "
              "library has no multi-GPU path (--gpus %d requested)" % args.gpus, file=sys.stderr)
        sys.exit(2)

    import torch
    import paper_1211_1645_amd.mpmc as mp

    torch.cuda.set_device(0)
    if args.copy_calibration:
        copy_calibration()
        return
    if args.workload == "positional":
        positional_bench(args)
        return
    if args.workload == "tau":
        tau_bench(args)
        return
    if args.workload == "scale":
        scale_bench(args)
        return
    if args.workload == "batch":
        batch_bench(args)
        return
    if args.workload == "pressure":
        pressure_bench(args)
        return
    if args.workload == "eos":
        eos_bench(args)
        return
    if args.workload == "tau-compare":
        tau_compare_bench(args)
        return
    if args.workload == "phases":
        phases_bench(args)
        return
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        box = mp.Box(N_DISKS, ETA, seed=args.seed, step_m=20, lattice="triangular",
                     schedule="fused" if args.tile else "auto", tile=args.tile,
                     stream=stream.cuda_stream)
        box.set_graphs(args.sweeps)  # one captured graph per benchmark step
        step_m, acc0 = tune_step(box)
        info = box.info()
        progress("step tuned (m = %d), schedule %s tile %d" % (step_m, info["schedule"], info["tile"]))
        # the measurements of a step (contact histogram, psi_6 and its field)
        # run on the box's measurement stream and overlap the next sweeps
        psi_dev = torch.zeros(max(args.steps, args.warmup, 1), 2, dtype=torch.float64,
                              device="cuda")
        for w in range(args.warmup):
            box.sweep(args.sweeps)
            box.measure_async(psi_dev[w], field=True)
        box.measure_wait()
        box.reset_contacts()
        torch.cuda.synchronize()

        t_before = box.info()
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(args.steps)]
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for s in range(args.steps):
            ev[s][0].record(stream)
            box.sweep(args.sweeps)
            ev[s][1].record(stream)
            box.measure_async(psi_dev[s], field=True)
        search_failed = box.measure_wait()
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t0
        t_after = box.info()
        progress("timed %d steps in %.3f s" % (args.steps, elapsed))
        if search_failed:
            raise RuntimeError("a psi_6 neighbour search was too short")
        psi_series = [complex(r, i) for r, i in psi_dev[:args.steps].cpu().tolist()]

    trials = t_after["trials"] - t_before["trials"]
    accepts = t_after["accepts"] - t_before["accepts"]
    sweep_ms = sum(a.elapsed_time(b) for a, b in ev) / (args.steps * args.sweeps)
    bytes_per = algorithmic_bytes_per_sweep(info["N"], info["M"])
    achieved_gbs = bytes_per / (sweep_ms * 1e-3) / 1e9
    trials_per_sweep = trials / (args.steps * args.sweeps)
    ops_per = trials_per_sweep * alu_ops_per_trial(info["N"], info["M"])
    achieved_tops = ops_per / (sweep_ms * 1e-3) / 1e12
    pressure = box.measure_pressure()
    overlaps, bad = box.validate()

    line = {
        "metric": "trial moves/s and psi6-decorrelation sweeps/s, 1024^2 disks eta=0.716",
        "value": trials / elapsed,
        "unit": "trial moves/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic (triangular-lattice start, Philox4x32-10 seed %d)" % args.seed,
        "config": {"workload": "plain MPMC, N=1024^2 hard disks, eta=0.716, triangular start, "
                               "1 trial per non-empty active cell, step tuned to ~30%% "
                               "acceptance (m=%d, d=%.4f sigma); step = %d sweeps + contact "
                               "histogram + psi6 field (measured on a second stream, overlapping the next "
                               "sweeps)" % (step_m, step_m / 256.0, args.sweeps),
                   "N": info["N"], "eta": ETA, "eta_eff": info["eta_eff"], "M": info["M"],
                   "w": info["w"], "n_trial": info["n_trial"], "step_m": step_m,
                   "sweeps_per_step": args.sweeps, "schedule": "fused" if info["schedule"] == 2
                   else "simple", "tile": info["tile"]},
        "sweeps_per_s": args.steps * args.sweeps / elapsed,
        "sweep_us": sweep_ms * 1e3,
        "acceptance": accepts / max(trials, 1),
        "trials_per_sweep": trials_per_sweep,
        "psi6_decorrelations_per_s": None,
        "psi6_tau_bound_at_this_point": stored_tau_bound(),
        "psi6_tau_at_paper_point": stored_tau(),
        "pressure_at_paper_point": stored_pressure(),
        "P_star_sample": pressure["P_star"],
        "abs_Psi6_mean": sum(abs(p) for p in psi_series) / len(psi_series),
        "validate": {"overlaps": overlaps, "bad": bad},
        "roofline": {"bound": "alu", "achieved": achieved_tops, "peak": ALU_PEAK_TOPS,
                     "unit": "TOP/s", "frac": achieved_tops / ALU_PEAK_TOPS,
                     "traffic": stored_traffic(),
                     "kernel": "k_fused (one sweep per launch)",
                     "algorithmic_ops_per_launch": ops_per,
                     "ops_per_trial": alu_ops_per_trial(info["N"], info["M"]),
                     "hbm": {"achieved": achieved_gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved_gbs / HBM_PEAK_GBS,
                             "algorithmic_bytes_per_launch": bytes_per},
                     "kernel_digest": kernel_source_digest()},
    }
    if not args.no_learned:
        line["learned_vs_uniform"] = {"sweep_cost_live": learned_speed(args.seed),
                                      "psi6_decorrelation": stored_tau_compare()}
        progress("learned comparison done")
    if not args.no_cpu_baseline:
        line["cpu_baseline"] = cpu_baseline(0, args.seed, step_m)
        progress("cpu baseline done")
    print(json.dumps(line))


if __name__ == "__main__":
    main()
