"""Benchmark of the level-set multigrid Crank-Nicolson step on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload batch64|star1025|torus257|disk65|serve|...]
                    [--precision 0|1] [--no-cpu-baseline] [--no-sequential]
                    [--requests R] [--load X] [--budget-gb G]

Workloads: batch64 (default) is 64 star domains of grid sizes 129^2 .. 1025^2
(10.8 M unknowns) stepped together, one launch per kernel and grid size, in
mixed precision (the headline value) and in FP64, beside the same domains
stepped one after another with the plain FP64 path; the oracle checks one
member of each grid size over every step run.  star1025 (FP64 by default),
torus257 and disk65 are single domains; serve is a seeded Poisson stream of
3-D simulations continuously batched under a memory budget, with p50/p99 step
latency, against the same requests run one after another.

Profiling helpers (they print text, not the benchmark line):
    python bench.py --copy-probe MIB          one plain device copy kernel over MIB MiB, 5 times
    python bench.py --trace-summary DIR       kernel table of a rocprofv3 --kernel-trace --stats run
    python bench.py --traffic FETCH WRITE COPY_FETCH COPY_WRITE [--copy-mib M]
                                              HBM bytes per launch of the finest-level smoother
                                              from four rocprofv3 --pmc runs; updates
                                              profiles/traffic.json

A step is one Crank-Nicolson step: Newton iterations whose linear systems are
solved by V-cycles, on synthetic seeded inputs already resident in HBM.  The
metric is V-cycle throughput, 2 (Ni + Ng) finest unknowns times the V-cycles
executed in the timed steps per second.  One JSON line is printed.
"""
import argparse
import hashlib
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

import lsmg_inputs as I  # noqa: E402

METRIC = "V-cycle unknowns·cycles/s at 1e-10 rel, mixed vs FP64; %HBM roofline; p99 step"
HBM_PEAK_GBS = 8000.0
WORKLOADS = {
    "star1025": dict(kind="star", dim=2, n=1025, coarsest=9, dt=1e-4, steps=100),
    "torus257": dict(kind="torus", dim=3, n=257, coarsest=9, dt=1e-4, steps=20),
    "disk65": dict(kind="disk", dim=2, n=65, coarsest=5, dt=1e-3, steps=10),
    # the paper's own efficiency test (section 4.2, Test 3): circle, s0 = 0, c0 = 10,
    # s_B = 1, dt = h, N = 256, W(2,1), 8 x 8 coarsest grid; box [-pi/2, pi/2]^2
    "paper3": dict(kind="paper_circle", dim=2, n=257, coarsest=9, dt=None, steps=20, box=I.PAPER_BOX, c0=10.0,
                   params=dict(nu1=2, nu2=1, cycle_gamma=2)),
    # single requests of the served stream (seed 0) stepped alone: request 22 (257^3, four
    # ellipsoids, smoothed union; its slow ghost modes set the serving p99) and request 10
    # (65^3, three ellipsoids) on its plain, creased union
    "request22": dict(kind="request", id=22, smooth=0.02, dim=3, n=257, coarsest=9, dt=1e-4, steps=160),
    "request10_creased": dict(kind="request", id=10, smooth=0.0, dim=3, n=65, coarsest=9, dt=1e-4, steps=20),
}


def levelset(w):
    if w["kind"] == "request":
        r = [q for q in I.serving_requests(24, seed=0) if q["id"] == w["id"]][0]
        assert r["n"] == w["n"] and r["dt"] == w["dt"]
        return I.ellipsoids(r["n"], r["centres"], r["semi"], smooth=w["smooth"])
    return {"star": I.star, "torus": I.torus, "disk": I.disk, "paper_circle": I.paper_circle}[w["kind"]](w["n"])


def box_of(w):
    return w.get("box", (-1.0, 1.0))


def dt_of(w):
    lo, hi = box_of(w)
    return w["dt"] if w["dt"] is not None else (hi - lo) / (w["n"] - 1)


def smoother_bytes(c2g, ni, ng, n, dim, P):
    """Algorithmic bytes of one colour launch of the collective smoother on a level:
    reads s and c at every active node (2P each), the correction (2P) at active
    nodes of the other colour, the right-hand side (2P) and the type byte at the
    updated nodes, and writes the correction (2P) at the updated nodes; in 2-D the
    colour-1 launch also copies each ghost's correction (index 4 + P read, P written).
    Returned for colour 0 and colour 1."""
    g = c2g.astype(np.int64)
    idx = [g % n, (g // n) % n] + ([g // (n * n)] if dim == 3 else [])
    col = sum(idx) & 1
    out = []
    for c in (0, 1):
        upd = int(np.sum(col[:ni] == c))
        other = int(np.sum(col != c))
        out.append(2 * P * (ni + ng) + 2 * P * other + (2 * P + 1) * upd + 2 * P * upd
                   + (ng * (4 + 2 * P) if (dim == 2 and c == 1) else 0))
    return out


def fused_sweep_bytes(c2g, ni, ng, n, P):
    """Algorithmic bytes of one fused 2-D sweep launch (both colours, k_smooth_rb):
    reads s, c and the type byte at every active node, the right-hand side at the
    inside nodes, the old correction (2P) at the black active nodes and the red
    ghosts (the red corrections reach the black half-sweep through LDS), writes the
    correction (2P) at every active node into the other copy, and snapshots each
    ghost's correction (index 4 + P read, P written)."""
    g = c2g.astype(np.int64)
    col = (g % n + (g // n) % n) & 1
    black_active = int(np.sum(col == 1))
    red_ghosts = int(np.sum(col[ni:] == 0))
    return ((2 * P + 1) * (ni + ng) + 2 * P * ni + 2 * P * (black_active + red_ghosts) + 2 * P * (ni + ng)
            + ng * (4 + 2 * P))


def source_hash():
    h = hashlib.sha256()
    for f in ("kernels.hip", "lsmg_dev.hpp"):
        h.update(open(os.path.join(ROOT, "paper_1902_07029_amd", "csrc", f), "rb").read())
    return h.hexdigest()[:16]


def load_traffic(kernel, workload, precision):
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    try:
        data = json.load(open(path))
        rec = data.get(f"{kernel}:{workload}:p{precision}")
        if rec and rec.get("source_hash") == source_hash():
            return rec["bytes_per_launch"]
    except Exception:
        return None
    return None


def host_cpu():
    """The host's CPU model and the number of cores this process may use."""
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    return {"model": model, "cores_available": ncpu}


def cpu_baseline(phi, dim, n, coarsest, dt, params, budget_s, gpu_states, label, max_steps=200, bc=0,
                 box=(-1.0, 1.0), c0=1.0):
    """The oracle (serial, one core) on the first steps of a domain of the workload,
    for about budget_s seconds; the steps it shares with gpu_states (gpu_states[k] is
    the compact GPU state after step k + 1) give a parity check of the GPU trajectory."""
    import oracle
    O = oracle.Hierarchy(phi, dim, n, *box, coarsest_n=coarsest, params=params, bc=bc)
    info = O.level_info(0)
    na = info["na"]
    s0, cc0 = I.initial_state(n, dim, 0.0, c0)
    W = O.to_compact(0, s0, cc0)
    sb = np.ones(info["ng"])
    cycles = 0
    worst = 0.0
    steps = 0
    t0 = time.perf_counter()
    while steps < max_steps:
        rc, W, st = O.newton_cn_step(W, dt, sb)
        if rc != 0:
            raise RuntimeError(f"oracle step failed with {rc}")
        cycles += st["vcycles"]
        if steps < len(gpu_states):
            G = gpu_states[steps]
            for blk in (slice(0, na), slice(na, 2 * na)):
                worst = max(worst, float(np.max(np.abs(G[blk] - W[blk])) / np.max(np.abs(W[blk]))))
        steps += 1
        if time.perf_counter() - t0 > budget_s and steps >= len(gpu_states):
            break
    el = time.perf_counter() - t0
    return dict(value=2 * na * cycles / el, unit="unknowns*cycles/s", cores=1, kind="oracle", host=host_cpu(),
                sample=f"first {steps} Crank-Nicolson steps of {label} ({cycles} V-cycles, {el:.1f} s, "
                       f"serial C, one host core)"), \
        dict(steps_checked=min(steps, len(gpu_states)), max_rel_err=worst, domain=label)


def _oracle_worker(job):
    """One host process of the all-cores baseline: the oracle stepping one domain for
    about budget seconds (module-level for the spawn start method)."""
    phi, dim, n, coarsest, dt, params, budget = job
    import oracle
    O = oracle.Hierarchy(phi, dim, n, coarsest_n=coarsest, params=params)
    info = O.level_info(0)
    s0, c0 = I.initial_state(n, dim)
    W = O.to_compact(0, s0, c0)
    sb = np.ones(info["ng"])
    cycles = steps = 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget:
        rc, W, st = O.newton_cn_step(W, dt, sb)
        if rc != 0:
            raise RuntimeError(f"oracle step failed with {rc}")
        cycles += st["vcycles"]
        steps += 1
    return 2 * info["na"] * cycles, time.perf_counter() - t0, steps, cycles


def cpu_baseline_pool(jobs_in, budget_s, label):
    """The oracle on every host core at once: one process per domain (the first
    domains of the workload), each for about budget_s seconds; the throughputs add."""
    import multiprocessing
    try:
        ncpu = len(os.sched_getaffinity(0))
    except AttributeError:
        ncpu = os.cpu_count() or 1
    workers = max(1, min(16, ncpu, len(jobs_in)))
    jobs = [j + (budget_s,) for j in jobs_in[:workers]]
    with multiprocessing.get_context("spawn").Pool(workers) as pool:
        res = pool.map(_oracle_worker, jobs)
    value = sum(u / el for u, el, _, _ in res)
    steps = sum(r[2] for r in res)
    cycles = sum(r[3] for r in res)
    return dict(value=value, unit="unknowns*cycles/s", cores=workers, kind="oracle", host=host_cpu(),
                sample=f"{workers} host processes at once, one domain each ({label}), "
                       f"{steps} Crank-Nicolson steps and {cycles} V-cycles in about {budget_s:.0f} s each")


def oracle_params(H):
    eff = H.params
    return {k: getattr(eff, k) for k in ("a", "d", "m_s", "m_c", "alpha", "beta", "tau_s", "nu1", "nu2",
                                         "ghost_c_new", "band_steps", "ghost_sweeps", "ghost_sweeps_coarse",
                                         "sweeps_lambda", "krylov_m")} | {"gamma": eff.cycle_gamma, "fmg": eff.fmg}


# ---------------------------------------------------------------- profiling helpers

SMOOTH_KERNELS = ("k_smooth_colour", "k_smooth_rb")


def _smooth_kernel(rows):
    """The finest level's smoother in a profile: the per-colour kernel where it ran
    (fused sweeps are used on the smaller levels only, or where the finest level
    itself is small), else the fused 2-D sweep."""
    for k in SMOOTH_KERNELS:
        if any(k in r["Kernel_Name"] for r in rows):
            return k
    raise SystemExit("no smoother dispatches in the profile")


def _csv_rows(directory, suffix):
    import csv
    import glob
    files = sorted(glob.glob(os.path.join(directory, "**", f"*{suffix}"), recursive=True))
    if not files:
        raise SystemExit(f"no *{suffix} under {directory}")
    rows = []
    for f in files:
        rows.extend(csv.DictReader(open(f)))
    return rows


def _short(name):
    name = name.replace("void ", "")
    head = name.split("(")[0]
    return head.replace("lsmg::", "")


def copy_probe(mib):
    """A plain elementwise copy (dst = -src) over mib MiB, five launches: the
    reference kernel of known size for scaling the FETCH_SIZE / WRITE_SIZE counters."""
    import torch
    n = mib * (1 << 20) // 4
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(5):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": n * 4, "launches": 5}))


def _finest(rows, key):
    """Rows of the finest-level smoother: the dispatches of the smoother kernel whose
    grid is at least half the largest grid (the next coarser level has about a quarter)."""
    kern = _smooth_kernel(rows)
    sm = [r for r in rows if kern in r["Kernel_Name"]]
    gmax = max(int(r[key]) for r in sm)
    return [r for r in sm if 2 * int(r[key]) >= gmax]


def trace_summary(directory):
    stats = _csv_rows(directory, "kernel_stats.csv")
    stats.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in stats)
    print(f"{'calls':>7} {'total ms':>9} {'share':>6} {'avg us':>8}  kernel")
    for r in stats[:20]:
        t = float(r["TotalDurationNs"])
        print(f"{int(r['Calls']):7d} {t / 1e6:9.3f} {100 * t / total:5.1f}% {float(r['AverageNs']) / 1e3:8.2f}  "
              f"{_short(r['Name'])}")
    trace = _csv_rows(directory, "kernel_trace.csv")
    for kern in SMOOTH_KERNELS:
        sm = [r for r in trace if kern in r["Kernel_Name"]]
        if not sm:
            continue
        by = {}
        for r in sm:
            g = int(r["Grid_Size_X"]) if "Grid_Size_X" in r else int(r["Grid_Size"])
            by.setdefault(g, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
        print(f"\n{kern} by grid size (threads), from the kernel trace:")
        for g in sorted(by, reverse=True):
            v = by[g]
            print(f"  grid {g:9d}  launches {len(v):6d}  avg {sum(v) / len(v) / 1e3:8.2f} us")
    kern = _smooth_kernel(trace)
    print(f"finest-level smoother: {kern}")
    fin = _finest(trace, "Grid_Size_X" if "Grid_Size_X" in trace[0] else "Grid_Size")
    d = [int(r["End_Timestamp"]) - int(r["Start_Timestamp"]) for r in fin]
    print(f"finest level: {len(d)} launches, average {sum(d) / len(d) / 1e3:.2f} us")


def trace_step(directory, k):
    """Kernels of one Crank-Nicolson step of a kernel trace: the dispatches from the
    k-th explicit-half launch (0-based; each step starts with one) to the next, with
    the step's span and the share of it during which the GPU ran a kernel."""
    rows = _csv_rows(directory, "kernel_trace.csv")
    for r in rows:
        r["_s"], r["_e"] = int(r["Start_Timestamp"]), int(r["End_Timestamp"])
    rows.sort(key=lambda r: r["_s"])
    starts = [i for i, r in enumerate(rows) if "k_explicit_half" in r["Kernel_Name"]]
    if k + 1 >= len(starts):
        raise SystemExit(f"the trace holds {len(starts)} step starts")
    seg = rows[starts[k]:starts[k + 1]]
    span = seg[-1]["_e"] - seg[0]["_s"]
    busy, last = 0, seg[0]["_s"]
    for r in seg:
        b = max(r["_s"], last)
        if r["_e"] > b:
            busy += r["_e"] - b
        last = max(last, r["_e"])
    by = {}
    for r in seg:
        key = _short(r["Kernel_Name"])
        c = by.setdefault(key, [0, 0])
        c[0] += 1
        c[1] += r["_e"] - r["_s"]
    print(f"step {k}: {len(seg)} dispatches, span {span / 1e3:.1f} us, GPU busy {busy / 1e3:.1f} us "
          f"({100.0 * busy / span:.0f} %)")
    print(f"{'calls':>7} {'total us':>10} {'avg us':>8}  kernel")
    for key, (c, t) in sorted(by.items(), key=lambda kv: -kv[1][1]):
        print(f"{c:7d} {t / 1e3:10.1f} {t / c / 1e3:8.2f}  {key}")


def _pmc_per_dispatch(directory, counter, finest):
    rows = [r for r in _csv_rows(directory, "counter_collection.csv") if r["Counter_Name"] == counter]
    if finest:
        rows = _finest(rows, "Grid_Size")
    vals = [float(r["Counter_Value"]) for r in rows]
    if not vals:
        raise SystemExit(f"no {counter} values under {directory}")
    return sum(vals) / len(vals), len(vals)


def _pmc_copy(directory, counter, mib):
    rows = [r for r in _csv_rows(directory, "counter_collection.csv") if r["Counter_Name"] == counter]
    big = max(float(r["Counter_Value"]) for r in rows)
    rows = [float(r["Counter_Value"]) for r in rows if float(r["Counter_Value"]) > 0.5 * big]
    kib = sum(rows) / len(rows)
    return (mib * 1024.0) / kib


def traffic(fetch_dir, write_dir, copy_fetch_dir, copy_write_dir, workload, precision, mib):
    f_kib, nf = _pmc_per_dispatch(fetch_dir, "FETCH_SIZE", True)
    w_kib, nw = _pmc_per_dispatch(write_dir, "WRITE_SIZE", True)
    sf = _pmc_copy(copy_fetch_dir, "FETCH_SIZE", mib)
    sw = _pmc_copy(copy_write_dir, "WRITE_SIZE", mib)
    fetch_b = f_kib * 1024 * sf
    write_b = w_kib * 1024 * sw
    kern = _smooth_kernel(_csv_rows(fetch_dir, "counter_collection.csv"))
    key = f"{kern[2:]}:{workload}:p{precision}"
    path = os.path.join(ROOT, "profiles", "traffic.json")
    data = json.load(open(path)) if os.path.exists(path) else {}
    data[key] = dict(bytes_per_launch=int(fetch_b + write_b), fetch_bytes=int(fetch_b), write_bytes=int(write_b),
                     fetch_kib_raw=f_kib, write_kib_raw=w_kib, copy_scale_fetch=sf, copy_scale_write=sw,
                     dispatches=[nf, nw], source_hash=source_hash())
    json.dump(data, open(path, "w"), indent=1, sort_keys=True)
    print(json.dumps({key: data[key]}))


def run_single(args):
    import torch
    from paper_1902_07029_amd import lsmg

    w = WORKLOADS[args.workload]
    prec = args.precision if args.precision is not None else 0
    bc = 1 if args.bc == "neumann" else 0
    params = lsmg.default_params(coarsest_n=w["coarsest"], precision=prec, bc=bc, fmg=args.fmg,
                                 fused_sweep=args.fused, krylov_m=args.krylov, **w.get("params", {}))
    phi_np = levelset(w)
    lo, hi = box_of(w)
    dt = dt_of(w)
    phi = torch.from_numpy(phi_np).cuda()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    H = lsmg.Hierarchy(phi, w["dim"], w["n"], lo, hi, params=params)
    torch.cuda.synchronize()
    build_ms = (time.perf_counter() - t0) * 1e3
    info = H.level_info(0)
    na, ni, ng = info["na"], info["ni"], info["ng"]
    unknowns = 2 * na
    s0, c0 = I.initial_state(w["n"], w["dim"], 0.0, w.get("c0", 1.0))

    def fresh_state():
        st = lsmg.State(H)
        st.set_grid(torch.from_numpy(s0).cuda(), torch.from_numpy(c0).cuda())
        return st

    st = fresh_state()
    for _ in range(args.warmup):
        st.step(dt)
    # timed region: K steps (V-cycles replayed as captured graphs)
    lat = []
    rho = []
    cycles = 0
    newton = 0
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        ts = time.perf_counter()
        _, stats = st.step(dt)
        lat.append(time.perf_counter() - ts)
        cycles += stats["vcycles"]
        newton += stats["newton_iters"]
        rho.append((stats["rho_geo"], stats["rho_last"]))
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    # kernel timing pass: the next K steps of the same run, every finest-level
    # smoother launch timed by its own dispatch events on the hierarchy's stream
    H.profile_start(lsmg.KERNEL_SMOOTH, 0)
    prof_t0 = time.perf_counter()
    for _ in range(args.steps):
        st.step(dt)
    torch.cuda.synchronize()
    prof_elapsed = time.perf_counter() - prof_t0
    launches, prof_ms = H.profile_stop()
    if launches == 0 and not H.tail_whole():
        raise RuntimeError("no timed launches of the dominant kernel")

    # roofline of the dominant kernel, the finest-level smoother: in 2-D pairs of
    # smoothing steps run as fused sweeps (both colours per launch), an odd step
    # as one launch per colour; the bytes per launch are averaged over one cycle
    P = 8 if prec == 0 else 4
    c2g0 = H.compact_to_grid(0).cpu().numpy()
    b0, b1 = smoother_bytes(c2g0, ni, ng, w["n"], w["dim"], P)
    eff = H.params
    if H.sweep_fused(0, prec):
        bf = fused_sweep_bytes(c2g0, ni, ng, w["n"], P)
        pairs = eff.nu1 // 2 + eff.nu2 // 2
        single = eff.nu1 % 2 + eff.nu2 % 2
        bytes_per_launch = (2 * pairs * bf + single * (b0 + b1)) / (2 * pairs + 2 * single)
        kname = "k_smooth_rb (finest level, both colours of a sweep)" if single == 0 else \
            "k_smooth_rb and k_smooth_colour (finest level)"
        tkey = "smooth_rb"
    else:
        bytes_per_launch = 0.5 * (b0 + b1)
        kname, tkey = "k_smooth_colour (finest level, one colour)", "smooth_colour"
    if launches:
        avg_s = prof_ms * 1e-3 / launches
        achieved = bytes_per_launch / avg_s / 1e9
        roofline = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                        frac=round(achieved / HBM_PEAK_GBS, 4),
                        traffic=load_traffic(tkey, args.workload, prec),
                        kernel=kname, launches=launches,
                        avg_us=round(avg_s * 1e6, 2), bytes_per_launch=int(bytes_per_launch),
                        timing_pass_ms_per_step=round(prof_elapsed * 1e3 / args.steps, 3))
    else:
        # every level fits the one-workgroup coarse tail: there is no smoother launch
        # to time, and a single workgroup is latency-bound by construction
        roofline = dict(bound="latency", achieved=None, peak=HBM_PEAK_GBS, unit="GB/s", frac=None, traffic=None,
                        kernel="coarse tail (the whole hierarchy runs in one workgroup)", launches=0)

    cpu = parity = None
    if not args.no_cpu_baseline:
        st2 = fresh_state()
        states = []
        for _ in range(args.parity_steps):
            st2.step(dt)
            states.append(st2.get().cpu().numpy())
        cpu, parity = cpu_baseline(phi_np, w["dim"], w["n"], w["coarsest"], dt, oracle_params(H),
                                   args.cpu_budget, states, f"{w['kind']} {w['n']}^{w['dim']}", bc=bc,
                                   box=(lo, hi), c0=w.get("c0", 1.0))

    lat_ms = np.array(lat) * 1e3
    return {
        "metric": METRIC,
        "value": unknowns * cycles / elapsed,
        "unit": "unknowns*cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": elapsed * 1e3 / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}_{'fp64' if prec == 0 else 'mixed'}" + ("_neumann" if bc else "")
                        + (f"_fmg{args.fmg}" if args.fmg else "") + (f"_krylov{args.krylov}" if args.krylov else ""),
            "boundary": "neumann ds/dn = 1" if bc else "dirichlet s = 1",
            "domain": w["kind"], "dim": w["dim"], "n": w["n"], "dt": dt, "coarsest": w["coarsest"],
            "box": [lo, hi], "c0": w.get("c0", 1.0),
            "unknowns": unknowns, "inside": ni, "ghost": ng, "levels": H.nlev,
            "cycle": f"{'VW'[H.params.cycle_gamma - 1]}({H.params.nu1},{H.params.nu2}) red-black, {H.params.ghost_sweeps} ghost sweeps "
                     f"({H.params.ghost_sweeps_coarse} where d dt/h^2 < {H.params.sweeps_lambda})",
            "fused_sweep_levels": [l for l in range(H.nlev) if H.sweep_fused(l, prec)],
            "linear_solve": (f"flexible GMRES({args.krylov}) preconditioned by one V-cycle" if args.krylov
                             else "V-cycles"),
            "build_ms": round(build_ms, 1),
        },
        "vcycles": cycles,
        "newton_iters": newton,
        # per step: geometric mean of all its convergence factors (the first cycle of each
        # Newton system included) and the factor of its last cycle
        "rho_geo_median": float(np.median([r[0] for r in rho])),
        "rho_last_median": float(np.median([r[1] for r in rho])),
        "solution_throughput": unknowns * args.steps / elapsed,
        "p50_step_ms": float(np.percentile(lat_ms, 50)),
        "p99_step_ms": float(np.percentile(lat_ms, 99)),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
    }


# Algorithmic HBM bytes per finest active node per V-cycle (the byte model of the
# kernels: four smoothing sweeps, the defect with the restriction, the
# prolongation and the cycle-end defect with its norm, with the coarse levels'
# share of 1/3 in 2-D and 1/7 in 3-D): 63 values of P bytes in 2-D, 55 in 3-D.
# The mixed cycle moves FP32 values and adds the FP64 refinement (defect and
# update, about 70 bytes per node).
def vcycle_bytes_per_node(dim, mixed):
    per = 63 if dim == 2 else 55
    return per * 4 + 70 if mixed else per * 8


def run_batch(args):
    """64 star domains of uneven grid sizes (129^2 .. 1025^2) stepped together, in
    mixed precision (the headline) and in FP64, against the same domains stepped one
    after another with the plain FP64 path.  For each precision: a parity pass of
    warmup + timed steps whose states of one member per grid size go to the oracle,
    then the timed run from the same initial states (checked to end bitwise where the
    parity pass ended), then a kernel timing pass."""
    import torch
    from paper_1902_07029_amd import lsmg

    doms = I.batch_domains(64, seed=0)
    dt = doms[0]["dt"]
    phis = [I.star(d["n"], **d["shape"]) for d in doms]
    sizes_all = sorted({d["n"] for d in doms})
    # parity members: the first domain of each grid size
    sample = [next(k for k, d in enumerate(doms) if d["n"] == n) for n in sizes_all]
    big = sample[-1]
    nsteps = args.warmup + args.steps
    precs = [1, 0] if args.precision is None else [args.precision]

    def build(prec):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Hs = [lsmg.Hierarchy(torch.from_numpy(phi).cuda(), 2, d["n"],
                             params=lsmg.default_params(coarsest_n=d["coarsest"], precision=prec,
                                                        fused_sweep=args.fused))
              for phi, d in zip(phis, doms)]
        B = lsmg.Batch(Hs)
        torch.cuda.synchronize()
        return Hs, B, (time.perf_counter() - t0) * 1e3

    def fresh_states(hs):
        out = []
        for H, d in zip(hs, doms):
            st = lsmg.State(H)
            s0, c0 = I.initial_state(d["n"], 2)
            st.set_grid(torch.from_numpy(s0).cuda(), torch.from_numpy(c0).cuda())
            out.append(st)
        return out

    runs = {}
    infos = None
    for prec in precs:
        Hs, B, build_ms = build(prec)
        opar = oracle_params(Hs[0])      # the members share their (resolved) parameters
        infos = [H.level_info(0) for H in Hs]
        na = np.array([inf["na"] for inf in infos], dtype=np.float64)
        # parity pass (the autotuner runs in its first step)
        states = fresh_states(Hs)
        traj = {k: [] for k in sample}
        for _ in range(nsteps):
            B.step(states, dt)
            for k in sample:
                traj[k].append(states[k].get().cpu().numpy())
        # timed run from the same initial states
        states = fresh_states(Hs)
        for _ in range(args.warmup):
            B.step(states, dt)
        lat = []
        cyc = np.zeros(len(doms))
        newton = 0
        torch.cuda.synchronize()
        t_start = time.perf_counter()
        for _ in range(args.steps):
            ts = time.perf_counter()
            _, stats = B.step(states, dt)
            lat.append(time.perf_counter() - ts)
            for k, stt in enumerate(stats):
                cyc[k] += stt["vcycles"]
                newton += stt["newton_iters"]
        torch.cuda.synchronize()
        elapsed = time.perf_counter() - t_start
        same = all(np.array_equal(states[k].get().cpu().numpy(), traj[k][-1]) for k in sample)
        # kernel timing pass: the smoother launches at the largest grid size.  A launch
        # covers the members of that size that are still solving, so each member is
        # credited with its own bytes for each cycle it ran: per cycle, nu1 + nu2
        # smoothing steps of its finest level (one launch per colour, or one fused launch)
        nmax = max(sizes_all)
        cyc_t = np.zeros(len(doms), dtype=np.int64)
        B.profile_start(lsmg.KERNEL_SMOOTH, nmax)
        for _ in range(args.steps):
            _, stt = B.step(states, dt)
            for k, sk in enumerate(stt):
                cyc_t[k] += sk["vcycles"]
        torch.cuda.synchronize()
        launches, prof_ms = B.profile_stop()
        tuning = {str(k): v for k, v in B.tuning().items()}
        P = 8 if prec == 0 else 4
        nsm = Hs[0].params.nu1 + Hs[0].params.nu2
        fused = B.sweep_fused(nmax, prec) and Hs[0].params.nu1 % 2 == 0 and Hs[0].params.nu2 % 2 == 0
        byts_full = byts_run = 0.0
        for k, (H, d, inf) in enumerate(zip(Hs, doms, infos)):
            if d["n"] == nmax:
                c2g0 = H.compact_to_grid(0).cpu().numpy()
                if fused:
                    per_step = fused_sweep_bytes(c2g0, inf["ni"], inf["ng"], d["n"], P)
                    byts_full += per_step
                else:
                    b0, b1 = smoother_bytes(c2g0, inf["ni"], inf["ng"], d["n"], 2, P)
                    per_step = b0 + b1
                    byts_full += 0.5 * (b0 + b1)
                byts_run += float(cyc_t[k]) * nsm * per_step
        kname = (f"k_smooth_rb (the {nmax}^2 levels of the batch still solving, both colours of a sweep)" if fused
                 else f"k_smooth_colour (the {nmax}^2 levels of the batch still solving, one colour)")
        avg_s = prof_ms * 1e-3 / max(launches, 1)
        byts = byts_run / max(launches, 1)
        achieved = byts / avg_s / 1e9 if launches else 0.0
        kern = dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(achieved / HBM_PEAK_GBS, 4),
                    traffic=load_traffic("smooth_rb" if fused else "smooth_colour", "batch64", prec),
                    kernel=kname, launches=launches, avg_us=round(avg_s * 1e6, 2), bytes_per_launch=int(byts),
                    bytes_all_members=int(byts_full))
        bpn = vcycle_bytes_per_node(2, prec == 1)
        vbytes = float(np.dot(na, cyc)) * bpn
        vcyc = dict(bound="hbm", achieved=round(vbytes / elapsed / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(vbytes / elapsed / 1e9 / HBM_PEAK_GBS, 4), bytes_per_node_cycle=bpn,
                    node_cycles=int(np.dot(na, cyc)),
                    model="algorithmic bytes per finest active node per V-cycle x nodes x cycles executed "
                          "/ timed wall time (all kernels, launch gaps and host work included)")
        lat_ms = np.array(lat) * 1e3
        # the same members as `groups` batches on their own streams, stepped concurrently
        grouped = None
        B = None
        if args.groups > 1:
            G = lsmg.BatchGroup(Hs, groups=args.groups)
            gst = fresh_states(Hs)
            for _ in range(args.warmup):
                G.step(gst, dt)
            gcyc = np.zeros(len(doms))
            glat = []
            torch.cuda.synchronize()
            tg = time.perf_counter()
            for _ in range(args.steps):
                ts = time.perf_counter()
                _, stats = G.step(gst, dt)
                glat.append(time.perf_counter() - ts)
                for k, stt in enumerate(stats):
                    gcyc[k] += stt["vcycles"]
            torch.cuda.synchronize()
            gel = time.perf_counter() - tg
            gsame = all(np.array_equal(gst[k].get().cpu().numpy(), traj[k][-1]) for k in sample)
            glat_ms = np.array(glat) * 1e3
            grouped = dict(groups=len(G.parts), domains_per_group=[len(p) for p in G.parts],
                           value=float(np.dot(2 * na, gcyc)) / gel, ms_per_step=gel * 1e3 / args.steps,
                           p50_step_ms=float(np.percentile(glat_ms, 50)), p99_step_ms=float(np.percentile(glat_ms, 99)),
                           vcycle_roofline_frac=round(float(np.dot(na, gcyc)) * bpn / gel / 1e9 / HBM_PEAK_GBS, 4),
                           timed_run_equals_checked_run=gsame)
            G.close()
            del G, gst
        runs[prec] = dict(value=float(np.dot(2 * na, cyc)) / elapsed, ms_per_step=elapsed * 1e3 / args.steps,
                          vcycles=int(cyc.sum()), newton_iters=newton,
                          solution_throughput=float(2 * na.sum()) * args.steps / elapsed,
                          p50_step_ms=float(np.percentile(lat_ms, 50)), p99_step_ms=float(np.percentile(lat_ms, 99)),
                          kernel_roofline=kern, vcycle_roofline=vcyc, build_ms=round(build_ms, 1),
                          tuning=tuning, timed_equals_parity_pass=same, concurrent_batches=grouped,
                          traj=traj)
        del states, Hs
        torch.cuda.synchronize()
    unk = np.array([2 * inf["na"] for inf in infos], dtype=np.float64)
    # the plain FP64 path, domain after domain
    seq = None
    if not args.no_sequential:
        H64 = [lsmg.Hierarchy(torch.from_numpy(phi).cuda(), 2, d["n"],
                              params=lsmg.default_params(coarsest_n=d["coarsest"], precision=0))
               for phi, d in zip(phis, doms)]
        st64 = fresh_states(H64)
        for st in st64:
            st.step(dt)
        nseq = max(1, min(args.steps, 5))
        cyc64 = np.zeros(len(doms))
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(nseq):
            for k, st in enumerate(st64):
                cyc64[k] += st.step(dt)[1]["vcycles"]
        torch.cuda.synchronize()
        el64 = time.perf_counter() - t1
        seq = dict(value=float(np.dot(unk, cyc64)) / el64, steps=nseq, ms_per_round=el64 * 1e3 / nseq,
                   solution_throughput=float(unk.sum()) * nseq / el64)
        del st64, H64
    # the oracle over the same steps of the parity members; its time on the largest
    # member is the one-core baseline
    cpu = parity = None
    if not args.no_cpu_baseline:
        import oracle
        par = []
        worst = {p: 0.0 for p in precs}
        for k in sample:
            d = doms[k]
            O = oracle.Hierarchy(phis[k], 2, d["n"], coarsest_n=d["coarsest"], params=opar)
            info = O.level_info(0)
            nak = info["na"]
            s0, c0 = I.initial_state(d["n"], 2)
            W = O.to_compact(0, s0, c0)
            sb = np.ones(info["ng"])
            errs = {p: [] for p in precs}
            ocyc = 0
            t0 = time.perf_counter()
            for j in range(nsteps):
                rc, W, stt = O.newton_cn_step(W, dt, sb)
                if rc != 0:
                    raise RuntimeError(f"oracle step failed with {rc} on member {k}")
                ocyc += stt["vcycles"]
                for p in precs:
                    G = runs[p]["traj"][k][j]
                    errs[p].append(max(float(np.max(np.abs(G[blk] - W[blk])) / np.max(np.abs(W[blk])))
                                       for blk in (slice(0, nak), slice(nak, 2 * nak))))
            el = time.perf_counter() - t0
            for p in precs:
                worst[p] = max(worst[p], max(errs[p]))
            par.append(dict(member=k, n=d["n"], steps=nsteps,
                            max_rel_err={("mixed" if p else "fp64"): max(errs[p]) for p in precs}))
            if k == big:
                cpu = dict(value=2 * nak * ocyc / el, unit="unknowns*cycles/s", cores=1, kind="oracle",
                           host=host_cpu(),
                           sample=f"batch member {k} (star {d['n']}^2): {nsteps} Crank-Nicolson steps, {ocyc} V-cycles "
                                  f"in {el:.1f} s, serial C, one host core")
        parity = dict(steps_checked=nsteps, timed_steps=args.steps, tolerance=1e-10,
                      max_rel_err={("mixed" if p else "fp64"): worst[p] for p in precs},
                      timed_run_equals_checked_run={("mixed" if p else "fp64"): runs[p]["timed_equals_parity_pass"]
                                                    for p in precs},
                      members=par)
    cpu_all = None
    if not args.no_cpu_baseline:
        jobs = [(phis[k], 2, doms[k]["n"], doms[k]["coarsest"], dt, opar) for k in range(len(doms))]
        cpu_all = cpu_baseline_pool(jobs, args.cpu_budget, "the batch's first domains, grids "
                                    + "/".join(str(doms[k]["n"]) for k in range(min(16, len(doms)))))
    head = runs[precs[0]]
    sizes = {}
    for d in doms:
        sizes[str(d["n"])] = sizes.get(str(d["n"]), 0) + 1

    def summary(r):
        return {k: v for k, v in r.items() if k != "traj"}

    out = {
        "metric": METRIC,
        "value": head["value"],
        "unit": "unknowns*cycles/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if precs[0] == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": "batch64" + ("" if args.precision is None else ("_fp64" if precs[0] == 0 else "_mixed")),
                   "precision": "mixed" if precs[0] == 1 else "fp64", "domains": len(doms), "grid_sizes": sizes,
                   "dt": dt, "coarsest": 9, "unknowns": int(unk.sum()), "cycle": "V(2,2) red-black"},
        "vcycles": head["vcycles"],
        "newton_iters": head["newton_iters"],
        "solution_throughput": head["solution_throughput"],
        "p50_step_ms": head["p50_step_ms"],
        "p99_step_ms": head["p99_step_ms"],
        "roofline": head["kernel_roofline"],
        "vcycle_roofline": head["vcycle_roofline"],
        "cpu_baseline": cpu,
        "cpu_baseline_all_cores": cpu_all,
        "parity": parity,
        "concurrent_batches": head["concurrent_batches"],
        "fp64_sequential": seq,
        "speedup_vs_fp64_sequential": (head["value"] / seq["value"]) if seq else None,
    }
    if len(precs) == 2:
        out["mixed_batched"] = summary(runs[1])
        out["fp64_batched"] = summary(runs[0])
        out["speedup_mixed_vs_fp64_batched"] = runs[1]["value"] / runs[0]["value"]
    else:
        out["run"] = summary(head)
    return out


def run_serve(args):
    """Serving: a seeded Poisson stream of 3-D simulations on unions of ellipsoids
    (grids 65^3 .. 257^3, 10-200 steps), continuously batched in mixed precision
    under a memory budget, against the same requests run one after another with the
    plain FP64 path."""
    import torch
    from paper_1902_07029_amd import lsmg
    from paper_1902_07029_amd.serve import Request, Server

    prec = args.precision if args.precision is not None else 1
    base = I.serving_requests(args.requests, rate=1.0, seed=0)
    # --creased: the unions as configuration 5 states them, the plain minimum of the
    # ellipsoids, instead of the smoothed union
    phis = [I.ellipsoids(r["n"], r["centres"], r["semi"], smooth=0.0 if args.creased else 0.02) for r in base]
    # the plain FP64 path, request after request: per-step time and cycles measured on
    # the first steps of each request, scaled to its number of steps
    p64 = lsmg.default_params(coarsest_n=9, precision=0)
    seq_time = 0.0
    seq_work = 0.0
    seq_failed = []
    for r, phi in zip(base, phis):
        H = lsmg.Hierarchy(torch.from_numpy(phi).cuda(), 3, r["n"], params=p64)
        H_na = H.level_info(0)["na"]
        st = lsmg.State(H)
        s0, c0 = I.initial_state(r["n"], 3)
        st.set_grid(torch.from_numpy(s0).cuda(), torch.from_numpy(c0).cuda())
        ok = st.step(r["dt"], check=False)[0] == lsmg.OK
        k = max(1, min(r["steps"], args.seq_steps))
        cyc = 0
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        for _ in range(k):
            if not ok:
                break
            rc, stt = st.step(r["dt"], check=False)
            ok = rc == lsmg.OK
            cyc += stt["vcycles"]
        el = time.perf_counter() - t1
        del st, H
        if not ok:
            # a request the method does not solve (a creased union) is left out of the comparison
            seq_failed.append(r["id"])
            continue
        seq_time += el / k * r["steps"]
        seq_work += 2 * H_na * cyc / k * r["steps"]
    seq_value = seq_work / seq_time
    # arrivals at `load` times the request rate the sequential path sustains
    rate = args.load * (len(base) - len(seq_failed)) / seq_time
    stream = I.serving_requests(args.requests, rate=rate, seed=0)
    reqs = [Request(r["id"], r["arrival"], 3, r["n"], r["steps"], r["dt"], phi) for r, phi in zip(stream, phis)]
    params = lsmg.default_params(coarsest_n=9, precision=prec)
    budget = int(args.budget_gb * (1 << 30)) if args.budget_gb else None
    # the served results of the requests whose whole oracle trajectories are stored
    checked = [] if args.creased else [rid for rid in (12, 17) if rid < len(reqs)]
    server = Server(params, budget_bytes=budget, keep_states=set(checked), krylov_m=args.krylov)
    rep = server.run(reqs)
    parity = None
    if checked:
        par = []
        for f in rep["finished"]:
            if f.get("id") not in checked or "state" not in f:
                continue
            g = np.load(os.path.join(ROOT, "tests", "golden", f"trajectory_serve_r{f['id']}.npz"))
            na, idx = int(g["na"]), g["idx"]
            W = f["state"]
            err = 0.0
            for b, blk in enumerate((slice(0, na), slice(na, 2 * na))):
                ref = g["norms"][-1, b]
                err = max(err, float(np.max(np.abs(W[blk][idx] - g["vals"][-1, b])) / ref),
                          abs(float(np.max(np.abs(W[blk]))) - ref) / ref)
            par.append(dict(request=f["id"], n=f["n"], steps=f["steps"], status=f["status"], max_rel_err=err,
                            against="stored oracle trajectory, 512 sampled nodes and the norms over all"))
        parity = dict(tolerance=1e-10, requests=par, max_rel_err=max((q["max_rel_err"] for q in par), default=None))
    # one core of the host running the oracle on the first steps of request 12 (129^3)
    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        # request 12 (129^3); on the creased unions request 19 (129^3), since the method
        # does not solve request 12 there
        r = base[19] if args.creased and len(base) > 19 else (base[12] if len(base) > 12 else base[0])
        # the solver parameters as the library resolves them in 3-D, read from a small hierarchy
        opar = oracle_params(lsmg.Hierarchy(torch.from_numpy(I.sphere(17)).cuda(), 3, 17, params=params))
        O = oracle.Hierarchy(phis[r["id"]], 3, r["n"], coarsest_n=9, params=opar)
        info = O.level_info(0)
        s0, c0 = I.initial_state(r["n"], 3)
        W = O.to_compact(0, s0, c0)
        sb = np.ones(info["ng"])
        cyc = k = 0
        t1 = time.perf_counter()
        while k < r["steps"] and time.perf_counter() - t1 < min(args.cpu_budget, 20.0):
            rc, W, stt = O.newton_cn_step(W, r["dt"], sb)
            cyc += stt["vcycles"]
            k += 1
        el = time.perf_counter() - t1
        cpu = dict(value=2 * info["na"] * cyc / el, unit="unknowns*cycles/s", cores=1, kind="oracle", host=host_cpu(),
                   sample=f"request {r['id']} ({r['n']}^3, {len(r['centres'])} ellipsoids): first {k} steps, "
                          f"{cyc} V-cycles in {el:.1f} s, serial C, one host core")
    # whole-cycle bytes over the served work: algorithmic bytes per finest active node per
    # V-cycle (3-D, this precision) x node-cycles, over the makespan and over the busy time
    bpn = vcycle_bytes_per_node(3, prec == 1)
    vbytes = rep["unknowns_cycles"] / 2 * bpn
    roofline = dict(bound="hbm", kind="whole V-cycle over the served work (byte model, all kernels and gaps)",
                    achieved=round(vbytes / rep["makespan_s"] / 1e9, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                    frac=round(vbytes / rep["makespan_s"] / 1e9 / HBM_PEAK_GBS, 4),
                    frac_busy=round(vbytes / max(rep["busy_s"], 1e-9) / 1e9 / HBM_PEAK_GBS, 4),
                    bytes_per_node_cycle=bpn, traffic=None)
    sizes = {}
    for r in base:
        sizes[str(r["n"])] = sizes.get(str(r["n"]), 0) + 1
    return {
        "metric": METRIC,
        "value": rep["throughput"],
        "unit": "unknowns*cycles/s",
        "n_gpus": 1,
        "steps": sum(r["steps"] for r in base),
        "warmup": 0,
        "ms_per_step": rep["makespan_s"] * 1e3 / max(sum(r["steps"] for r in base), 1),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == 0 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"serve{args.requests}_{'fp64' if prec == 0 else 'mixed'}"
                               + (f"_krylov{args.krylov}" if args.krylov else "") + ("_creased" if args.creased else ""),
                   "requests": len(reqs), "grid_sizes": sizes, "arrival_rate_per_s": rate, "load": args.load,
                   "budget_bytes": server.budget, "dt": 1e-4, "coarsest": 9},
        "p50_step_ms": rep["p50_step_ms"],
        "p99_step_ms": rep["p99_step_ms"],
        # requests whose first step took more than 60 V-cycles and that then ran alone
        # with Krylov solves (--krylov M; their steps are not in busy_s, which counts
        # the batch's advance calls)
        "krylov_lane": dict(m=args.krylov, requests=rep["krylov_lane"]) if args.krylov else None,
        "completed": rep["completed"],
        "failed": [dict(id=f["id"], status=f.get("status")) for f in rep["finished"] if f.get("status") != 0],
        "makespan_s": rep["makespan_s"],
        "ticks": rep["ticks"],
        "advance_calls": rep["advance_calls"],
        "busy_s": rep["busy_s"],
        "busy_throughput": rep["busy_throughput"],
        "busy_speedup_vs_fp64_sequential": rep["busy_throughput"] / seq_value,
        "mean_members": rep["mean_members"],
        "max_members": rep["max_members"],
        "mean_queue_wait_s": rep["queue_wait_s"],
        "solution_throughput": rep["solution_throughput"],
        "fp64_sequential": dict(value=seq_value, time_s=seq_time, steps_measured_per_request=args.seq_steps,
                                failed_requests=seq_failed),
        "speedup_vs_fp64_sequential": rep["throughput"] / seq_value,
        "est_vs_actual_bytes": max(f["bytes"] / f["est_bytes"] for f in rep["finished"] if "bytes" in f),
        "roofline": roofline,
        "cpu_baseline": cpu,
        "parity": parity,
    }


def run_prepare(args):
    """Input preparation of a 1025^2 domain (sections 2 and 3.3): a pixel mask (the
    necklace of discs) made a level set, re-initialised, and non-constant initial
    data extrapolated to the ghosts.  Throughput in grid-node iterations per second
    of the re-initialisation, whose step is the dominant kernel."""
    import torch
    from paper_1902_07029_amd import lsmg
    import oracle
    n, dim, iters = 1025, 2, 200
    h = 2.0 / (n - 1)
    nn = n * n
    mask = torch.from_numpy(I.necklace_mask(n).astype(np.uint8)).cuda()
    phi_mask = lsmg.levelset_from_mask(mask, dim, n, 8)
    x, y = I.grid_points(n, 2)
    q = torch.from_numpy(np.ascontiguousarray(I.s_exact(x, y, 0.0))).cuda()
    for _ in range(args.warmup):
        lsmg.reinitialize(phi_mask.clone(), dim, n, iters)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ms_reinit = []
    for _ in range(args.steps):
        phi = phi_mask.clone()
        ev0.record()
        lsmg.reinitialize(phi, dim, n, iters)
        ev1.record()
        torch.cuda.synchronize()
        ms_reinit.append(ev0.elapsed_time(ev1))
    t0 = time.perf_counter()
    for _ in range(args.steps):
        lsmg.extrapolate(phi, q.clone(), dim, n, 40)
    torch.cuda.synchronize()
    ms_extrap = (time.perf_counter() - t0) * 1e3 / args.steps
    per_call = float(np.median(ms_reinit))
    value = nn * iters / (per_call * 1e-3)
    # one re-initialisation step reads phi (its four neighbours come from the same
    # rows), phi0, the near flag and the target D, and writes phi: 8 + 8 + 1 + 8 + 8 bytes
    bytes_per_iter = nn * 33
    achieved = bytes_per_iter * iters / (per_call * 1e-3) / 1e9
    cpu = None
    if not args.no_cpu_baseline:
        # the oracle's own level set of the same mask (no input from the GPU path)
        phi_np = oracle.levelset_from_mask(I.necklace_mask(n).astype(np.uint8), dim, n, 8)
        k = 0
        t1 = time.perf_counter()
        while time.perf_counter() - t1 < min(args.cpu_budget, 10.0):
            phi_np = oracle.reinitialize(phi_np, dim, n, h, 50)
            k += 50
        el = time.perf_counter() - t1
        cpu = dict(value=nn * k / el, unit="node*iterations/s", cores=1, kind="oracle",
                   sample=f"{k} re-initialisation steps on the 1025^2 necklace level set ({el:.1f} s, serial C)")
    return {
        "metric": "level-set re-initialisation node*iterations/s (input preparation)",
        "value": value, "unit": "node*iterations/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": per_call, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": "prepare1025", "n": n, "reinit_iterations": iters, "extrapolation_iterations": 40,
                   "mask": "necklace of 8 discs", "heat_steps": 8},
        "extrapolate_ms": ms_extrap,
        "roofline": dict(bound="hbm", achieved=round(achieved, 1), peak=HBM_PEAK_GBS, unit="GB/s",
                         frac=round(achieved / HBM_PEAK_GBS, 4), traffic=None,
                         kernel="k_reinit_step (whole re-initialisation call, events on the stream)",
                         bytes_per_launch=bytes_per_iter, avg_us=round(per_call * 1e3 / iters, 2)),
        "cpu_baseline": cpu,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", default="batch64", choices=sorted(WORKLOADS) + ["batch64", "serve", "prepare1025"],
                    help="paper3: the paper's Test 3 with its W(2,1) cycle (section 4.2)")
    ap.add_argument("--requests", type=int, default=24, help="serve: number of requests")
    ap.add_argument("--load", type=float, default=2.0,
                    help="serve: arrival rate as a multiple of the sequential FP64 request rate")
    ap.add_argument("--seq-steps", type=int, default=6, help="serve: steps timed per request on the FP64 path")
    ap.add_argument("--budget-gb", type=float, default=None, help="serve: memory budget (default 80%% of free)")
    ap.add_argument("--precision", type=int, default=None, choices=(0, 1),
                    help="0 = FP64, 1 = mixed (default: single domains FP64; batch64 both, mixed the headline)")
    ap.add_argument("--bc", default="dirichlet", choices=("dirichlet", "neumann"),
                    help="star1025 / torus257 / disk65: boundary condition for s (section 3.6 for Neumann)")
    ap.add_argument("--fmg", type=int, default=0, choices=(0, 1, 2),
                    help="single domains: full multigrid as the first iteration of the first (1) or every (2) "
                         "linear solve of a step")
    ap.add_argument("--krylov", type=int, default=0,
                    help="single domains: the linear solves by flexible GMRES(M) preconditioned by one V-cycle; "
                         "serve: the Krylov lane for requests whose first step needs more than 60 V-cycles "
                         "(0: plain V-cycles)")
    ap.add_argument("--creased", action="store_true",
                    help="serve: the plain (creased) unions of ellipsoids instead of the smoothed ones")
    ap.add_argument("--fused", type=int, default=1, choices=(0, 1),
                    help="2-D: both colours of a smoothing sweep in one launch (1) or one launch per colour (0)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-sequential", action="store_true", help="batch64: skip the sequential FP64 comparison")
    ap.add_argument("--groups", type=int, default=3,
                    help="batch64: also step the domains as this many concurrent batches on their own streams "
                         "(1 = off)")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--parity-steps", type=int, default=6)
    ap.add_argument("--copy-probe", type=int, metavar="MIB")
    ap.add_argument("--trace-summary", metavar="DIR")
    ap.add_argument("--trace-step", type=int, metavar="K",
                    help="with --trace-summary: also the kernels of the K-th step of the trace (0-based)")
    ap.add_argument("--traffic", nargs=4, metavar=("FETCH", "WRITE", "COPY_FETCH", "COPY_WRITE"))
    ap.add_argument("--copy-mib", type=int, default=512)
    args = ap.parse_args()
    if args.trace_summary:
        trace_summary(args.trace_summary)
        if args.trace_step is not None:
            print()
            trace_step(args.trace_summary, args.trace_step)
        return None
    if args.traffic:
        return traffic(*args.traffic, args.workload, args.precision or 0, args.copy_mib)
    if args.copy_probe:
        return copy_probe(args.copy_probe)
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for {args.gpus}); sharding over several GPUs "
              "is designed but not built", file=sys.stderr)
        sys.exit(2)
    import torch
    torch.cuda.set_device(0)
    if args.workload == "batch64":
        out = run_batch(args)
    elif args.workload == "serve":
        out = run_serve(args)
    elif args.workload == "prepare1025":
        out = run_prepare(args)
    else:
        out = run_single(args)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
