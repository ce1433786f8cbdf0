#!/usr/bin/env python3
"""Benchmark of the two-phase SEM-LBM time step on one MI355X.

Metric: FP64 node-updates/s.  One node-update advances one unique global GLL node by
one full time step (collision + three SSP-RK3 streaming stages, all populations).
Default workload: c4, the D3Q19 droplet on a sphere (cubed-sphere shell of 24,000 curved
hexes in a 128^3 box, N=5, about 3.06 M global nodes), the largest single-GPU
configuration; the default line also carries c2, c2-XL, batched-stepping and serving
objects and the oracle's CPU rate on c4.  All inputs are seeded and synthetic and
resident in device memory before the timed region.

Prints one JSON line (see the "value", "roofline", "fp64" and "cpu_baseline" keys).
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E
FP64_PEAK_TFLOPS = 78.6  # MI355X dense FP64, vector and matrix alike


def algorithmic_bytes(kind: str, Q: int, d: int, Ng: int, Nl: int, Ni: int = 0) -> float:
    """Bytes one launch of a kernel kind reads and writes at their minimum size: each FP64
    array it takes or produces counted once (arrays of global nodes at Ng, of local nodes at
    Nl; index tables are not counted).  The per-local-copy partial sums that pass from an
    element kernel to a node kernel are this kernel's inputs or outputs and are counted,
    at one value per local copy; the whole-step model (step_model_bytes) does not count them.

    Ni: global nodes strictly inside an element that the unfused element kernels finish
    themselves (one local copy each); the node kernels mu, collide and rk then run over the
    other Ns = Ng - Ni nodes, whose Nb = Nl - Ni local copies carry partial sums."""
    ng = d * (d + 1) // 2
    Ns, Nb = Ng - Ni, Nl - Ni
    per = {
        # reads rho (Ng), metric G (ng*Nl); interior: 1/M (Ni) -> mu (Ni); others -> partials (Nb)
        "lap": Ng + ng * Nl + 2 * Ni + Nb,
        # reads the Laplacian partials (Nb), rho, 1/M; writes mu (Ns nodes)
        "mu": Nb + 3 * Ns,
        # reads rho, mu, metric Ja; interior: f (Q), 1/M -> f* (Q); others -> 2d gradient partials
        "grad": 2 * Ng + d * d * Nl + (2 * Q + 1) * Ni + 2 * d * Nb,
        # reads 2d gradient partials (Nb), f (Q), rho, 1/M; writes f* (Q) (Ns nodes)
        "collide": 2 * d * Nb + (2 * Q + 2) * Ns,
        # reads g (Q-1 populations; interior also the rest population), rho, mu, metric Ja;
        # interior: g0 (2Q/3 on average over the three stages: stage 1's input is g0 itself),
        # 1/M -> g' (Q) and rho; others -> Q-1 residual partials (Nb)
        "stream": (Q - 1) * Ng + 2 * Ng + d * d * Nl + (1 + (2 * Q) / 3.0 + 1 + Q + 1) * Ni + (Q - 1) * Nb,
        # reads Q-1 residual partials (Nb), g (Q), g0 (2Q/3 on average), 1/M; writes Q
        # populations and rho (Ns nodes)
        "rk": (Q - 1) * Nb + (Q + (2 * Q) / 3.0 + 1 + Q + 1) * Ns,
        # fused path: each kernel finishes the previous pass's summation itself
        # A: Laplacian sum, rho, 1/M -> mu; metric Ja -> 2d gradient sums
        "f_mu_grad": 4 * Ng + d * d * Nl + 2 * d * Ng,
        # B: 2d gradient sums, 1/M, f (Q), rho, mu -> f* (Q); Ja -> Q-1 residual sums
        "f_collide_stream": (2 * d + 1 + Q + 2 + Q + (Q - 1)) * Ng + d * d * Nl,
        # C: Q-1 residual sums, 1/M, g (Q), g0 (2Q/3 on average over the three stages)
        #    -> g' (Q), rho; metric G -> Laplacian sum
        "f_rk_lap": ((Q - 1) + 1 + Q + (2 * Q) / 3.0 + Q + 2) * Ng + ng * Nl,
        # D: Laplacian sum, rho, 1/M, g (Q), Ja -> Q-1 residual sums
        "f_mu_stream": (3 + Q + (Q - 1)) * Ng + d * d * Nl,
    }[kind]
    return 8.0 * per


def step_model_bytes(Q: int, d: int, Ng: int, Nl: int) -> float:
    """Whole-step model: 9Q population doubles per node plus three stages of geometry
    (8 doubles per local node in 2-D, 16 in 3-D) and 4 scalars per node."""
    Gd = 8 if d == 2 else 16
    return 8.0 * (9 * Q * Ng + 3 * (Gd * Nl + 4 * Ng))


def make_case(name: str):
    from synth import cases
    return cases.CASES[name]()


def host_threads() -> int:
    """Host threads the oracle may use: this process's CPU share (affinity mask), capped by
    OMP_NUM_THREADS when that is set."""
    n = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else (os.cpu_count() or 1)
    env = os.environ.get("OMP_NUM_THREADS", "")
    if env.isdigit() and int(env) > 0:
        n = min(n, int(env))
    return max(1, n)


def cpu_baseline(case, budget_1: float = 15.0, budget_all: float = 6.0):
    """The C oracle timed on this host on a bounded sample of the workload: whole time
    steps at one thread until about budget_1 seconds have passed (at least one), then at
    every host thread this process may use (its OpenMP element and node loops; the sums
    stay sequential, so the results do not depend on the thread count) for about
    budget_all seconds.  `value` is the all-thread rate."""
    from oracle import Oracle, set_threads
    o = Oracle(case)
    o.init_tanh()

    def timed(budget):
        n, t0 = 0, time.perf_counter()
        chunk = 1
        while True:
            o.step(chunk)
            n += chunk
            el = time.perf_counter() - t0
            if el >= budget:
                return n, el
            # the next chunk ends near the budget (steps cost the same)
            chunk = max(1, min(4 * chunk, int((budget - el) / (el / n))))

    set_threads(1)
    n1, dt1 = timed(budget_1)
    nth = set_threads(host_threads())
    nn, dtn = timed(budget_all)
    set_threads(1)
    ng = case.mesh.n_global
    return dict(value=ng * nn / dtn, unit="node-updates/s", cores=nth, kind="oracle",
                sample=f"{case.name}: {n1} full time step(s) of the C oracle at 1 thread "
                       f"({dt1:.1f} s wall), then {nn} at {nth} threads ({dtn:.1f} s wall)",
                seconds_per_step=dtn / nn,
                single_core={"value": ng * n1 / dt1, "cores": 1, "seconds_per_step": dt1 / n1},
                host_nproc=os.cpu_count(), host_cpu_share=host_threads())


def kernels_sha256(csrc: str | None = None) -> str:
    """SHA-256 over the device sources (kernels.hpp, kernels*.hip, internal.hpp) in name
    order, with // comments and blank lines removed (comment edits leave it unchanged)."""
    import hashlib
    csrc = csrc or os.path.join(ROOT, "paper_2609_00535_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.startswith("kernels") or name == "internal.hpp":
            for line in open(os.path.join(csrc, name), encoding="utf-8"):
                code = line.split("//", 1)[0].rstrip()
                if code:
                    h.update(code.encode() + b"\n")
    return h.hexdigest()


def traffic_from_profiles(workload: str, kind: str):
    """HBM bytes per launch of the dominant kernel from the committed PMC summary, if it
    was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_sha256") != kernels_sha256():
        return None
    per = rec.get("bytes_per_launch", {})
    v = per.get(kind)
    return float(v) if v is not None else None


def fp64_from_profiles(workload: str):
    """FP64 flops per launch of each kernel kind from the committed instruction-counter
    summary, if it was taken on the current kernel source (else None)."""
    path = os.path.join(ROOT, "profiles", f"fp64_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("kernels_sha256") != kernels_sha256():
        return None
    return {k: float(v) for k, v in rec.get("flops_per_launch", {}).items()}


def fp64_point(flops: dict | None, prof: dict, profile_steps: int, ms_per_step: float,
               dom: str, avg_launch_ms: float, model_bytes: float):
    """The step's FP64 rate against the FP64 peak: counted flops per launch of every kernel
    kind times its launches per step (from the profiled steps), over the step time."""
    if not flops or any(k not in flops for k in prof):
        return None
    per_step = sum(flops[k] * nl / profile_steps for k, (_, nl) in prof.items())
    tf = per_step / (ms_per_step * 1e-3) / 1e12
    tf_dom = flops[dom] / (avg_launch_ms * 1e-3) / 1e12
    return {"achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": tf / FP64_PEAK_TFLOPS,
            "flops_per_step": per_step, "flop_per_model_byte": per_step / model_bytes,
            "kernel": dom, "kernel_achieved": tf_dom, "kernel_frac": tf_dom / FP64_PEAK_TFLOPS,
            "source": "rocprofv3 FP64 VALU instruction counters (profiles/fp64_<workload>.json); "
                      "all 64 lanes of each instruction counted, so an upper bound"}


def copy_calibration(torch, mib: int, reps: int = 3):
    """A plain streaming kernel of known size (y = -x over mib MiB of FP64) for scaling the
    HBM byte counters of a profiler pass: each launch reads and writes mib MiB."""
    n = (mib << 20) // 8
    x = torch.ones(n, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    torch.cuda.synchronize()
    for _ in range(reps):
        torch.neg(x, out=y)
    torch.cuda.synchronize()
    return {"copy_calibration": {"kernel": "elementwise neg (FP64)", "bytes_read": n * 8,
                                 "bytes_written": n * 8, "launches": reps}}


def batch_bench(P, torch, n_req: int, steps: int, warmup: int = 40, seed: int = 5):
    """Batched stepping: n_req solves of the request mix (see serving_bench) advanced as one
    batch, against the same solves stepped one at a time.  The warm-up covers the launch
    shape autotuner (four steps per candidate shape of each group).  Both timings are HIP
    events on the solves' stream around graph-replayed steps, inputs resident."""
    from synth import cases
    reqs = cases.request_stream(n_req, seed=seed)
    stream = torch.cuda.Stream()
    ev = lambda: torch.cuda.Event(enable_timing=True)
    with torch.cuda.stream(stream):
        ss = []
        for r in reqs:
            s = P.Solve(cases.request_case(r), stream=stream)
            s.init_tanh()
            ss.append(s)
        ng = sum(s.Ng for s in ss)
        b = P.Batch(stream)
        for s in ss:
            b.add(s)
        b.step(warmup)
        torch.cuda.synchronize()
        t0, t1 = ev(), ev()
        t0.record(stream)
        b.step(steps)
        t1.record(stream)
        t1.synchronize()
        ms_batch = t0.elapsed_time(t1) / steps
        shapes = b.shapes()
        del b
        # one at a time: every solve's own graph-replayed steps
        plain_ms = 0.0
        p_steps = max(10, steps // 5)
        by_class = {}
        for r, s in zip(reqs, ss):
            s.step(2)
            a, z = ev(), ev()
            a.record(stream)
            s.step(p_steps)
            z.record(stream)
            z.synchronize()
            ms1 = a.elapsed_time(z) / p_steps
            plain_ms += ms1
            key = f"{r['geom']} {r['nx']}x{r['ny']} N={r['N']}"
            c = by_class.setdefault(key, [0, 0.0, 0])
            c[0] += 1
            c[1] += ms1
            c[2] += s.Ng
    return {
        "members": n_req, "steps": steps, "warmup": warmup, "n_global_total": int(ng),
        "ms_per_step": ms_batch, "node_updates_per_s": ng / (ms_batch * 1e-3),
        "plain_ms_per_step_all_members": plain_ms,
        "batched_over_plain": plain_ms / ms_batch,
        # the one-at-a-time stepper's rate by request class: members, us per step of one
        # member, node-updates/s (the batch's rate is node_updates_per_s above)
        "plain_by_class": {k: {"members": v[0], "us_per_step": 1e3 * v[1] / v[0],
                               "node_updates_per_s": v[2] / (v[1] * 1e-3)}
                           for k, v in sorted(by_class.items())},
        "groups": [{"lattice": f"D{g['dim']}Q{g['lattice']}", "N": g["N"],
                    "fused": g["fused"], "members": g["members"], "elements": g["elements"],
                    "chosen": g["shapes"][g["chosen"]], "timed": g["measured"],
                    "candidates": g["shapes"]} for g in shapes],
    }


def serving_bench(P, torch, n_req: int, max_steps: int, check_every: int = 100,
                  ke_stop: float = 1e-20, max_slots: int = 256, seed: int = 5,
                  arena_mb: int = 8192, poisson: bool = True, plain: bool = True):
    """Request sweep c5 (reduced): n_req droplet requests (flat or cylinder wall, N in {4,6,8},
    theta ~ U[30,150], R ~ U[10,30]) run to KE_max < ke_stop or max_steps.

    Three runs of the same request list: (1) the plain stepper, one solve at a time with
    the same KE check cadence; (2) the continuous-batching server with every request
    submitted at once (throughput); (3) the server under Poisson arrivals at 0.7x the
    measured batched capacity (latency p50/p99 from arrival to retirement)."""
    import numpy as np

    from synth import cases
    reqs = cases.request_stream(n_req, seed=seed)
    cs = []
    for r in reqs:
        c = cases.request_case(r)
        c.steps = max_steps
        cs.append(c)
    stream = torch.cuda.Stream()
    # (1) plain stepper
    t0 = time.perf_counter()
    plain_steps = []
    t_note = time.perf_counter()
    with torch.cuda.stream(stream):
        for ci, c in enumerate(cs if plain else []):
            if time.perf_counter() - t_note > 20.0:
                t_note = time.perf_counter()
                print(f"[serve] plain stepper: {ci}/{len(cs)} requests, {t_note - t0:.0f} s", file=sys.stderr,
                      flush=True)
            s = P.Solve(c, stream=stream)
            s.init_tanh()
            n = 0
            while n < max_steps:
                s.step(check_every)
                n += check_every
                ke, _ = s.kinetic_energy()
                if not (ke <= 1.0) or ke < ke_stop:
                    break
            plain_steps.append(n)
            del s
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t0

    def run_server(arrivals):
        srv = P.Server(arena_bytes=arena_mb << 20, max_slots=max_slots, check_every=check_every,
                       ke_stop=ke_stop, max_steps=max_steps, stream=stream)
        ids = [None] * len(cs)
        order = np.argsort(arrivals)
        k = 0
        t_start = srv.clock()
        pending = 1
        t_note = t_start
        while k < len(cs) or pending > 0:
            now = srv.clock() - t_start
            if srv.clock() - t_note > 20.0:
                t_note = srv.clock()
                print(f"[serve] server: {k}/{len(cs)} submitted, {pending} pending, {now:.0f} s",
                      file=sys.stderr, flush=True)
            while k < len(cs) and arrivals[order[k]] <= now:
                ids[order[k]] = srv.submit(cs[order[k]])
                k += 1
            pending = srv.tick()
            if pending == 0 and k < len(cs):
                time.sleep(max(0.0, arrivals[order[k]] - (srv.clock() - t_start)))
        t_total = srv.clock() - t_start
        res = [srv.poll(i) for i in ids]
        lat = np.array([r.t_done - r.t_arrive for r in res])
        ok = sum(1 for r in res if r.status == 0)
        steps = [r.steps for r in res]
        theta = [r.theta_deg for r in res]
        status = [r.status for r in res]
        del srv
        return t_total, lat, ok, steps, theta, status

    with torch.cuda.stream(stream):
        t_batch, lat_b, ok_b, steps_b, theta_b, status_b = run_server(np.zeros(len(cs)))
        cap = len(cs) / t_batch
        if poisson:
            arr = np.array([r["t_arrive"] for r in reqs]) / (0.7 * cap)
            t_pois, lat_p, ok_p, _, _, _ = run_server(arr - arr.min())
        else:
            t_pois, lat_p, ok_p = float("nan"), np.array([float("nan")]), 0
    # retired by the KE criterion: finished without error before the step cap (a diverged
    # request also stops early, with a nonzero status)
    stopped_ke = sum(1 for s_, st in zip(steps_b, status_b) if s_ < max_steps and st == 0)
    st_arr = np.array(steps_b)
    per_req = [{"geom": r["geom"], "nx": r["nx"], "ny": r["ny"], "N": r["N"],
                "theta_deg": round(r["theta_deg"], 2), "steps": int(n), "status": int(st)}
               for r, n, st in zip(reqs, steps_b, status_b)]
    diverged = [q for q in per_req if q["status"] != 0]
    return {
        "metric": "batched sweep solves/s",
        "requests": len(cs), "max_steps": max_steps, "check_every": check_every,
        "ke_stop": ke_stop, "max_slots": max_slots,
        "batched_solves_per_s": len(cs) / t_batch,
        "plain_solves_per_s": len(cs) / t_plain if plain else None,
        "batched_over_plain": t_plain / t_batch if plain else None,
        "plain_s": t_plain if plain else None, "batched_s": t_batch,
        "saturated_latency_s": {"p50": float(np.percentile(lat_b, 50)),
                                "p99": float(np.percentile(lat_b, 99))},
        "poisson_0p7": {"rate_per_s": 0.7 * cap, "makespan_s": t_pois,
                        "latency_p50_s": float(np.percentile(lat_p, 50)),
                        "latency_p99_s": float(np.percentile(lat_p, 99)), "ok": ok_p},
        "ok": ok_b, "retired_by_ke": stopped_ke, "failed": diverged, "arena_mb": arena_mb,
        "steps_to_retire": {"min": int(st_arr.min()), "p50": float(np.percentile(st_arr, 50)),
                            "max": int(st_arr.max())},
        "plain_steps_match": ([int(a) for a in plain_steps] == [int(b) for b in steps_b]) if plain else None,
        "per_request": per_req if len(per_req) <= 64 else None,
        "plain_total_steps": int(sum(plain_steps)), "batched_total_steps": int(sum(steps_b)),
        "theta_err_deg_median": float(np.nanmedian(np.abs(np.array(theta_b) -
                                                           np.array([c.theta_deg for c in cs])))),
    }


def paper_runs(P, torch, kind: str, steps: int, every: int):
    """The paper's parasitic-current tests in its own settings, in lattice units; every
    run of a kind steps as one batch, KE_max of each is read every `every` steps and, for
    the walled caps, the contact angle at the end.  Each case carries the viscosity nu of its
    Laplace number and the library sets tau = nu / (cs^2 dt) at the time step; the isolated
    set runs at one time step (the smallest of its automatic ones).
      flat:     Sec. 3.1, N = 16, 16x8 elements, La = 122, equilibrium caps at 30-150 deg;
      curved:   Sec. 3.2, N = 11, circular wall on a 256-element O-grid, La = 341, equilibrium
                caps at 30-150 deg;
      curved-fine: the same on a 4x finer O-grid (1,024 elements);
      flat-orders: the 60-degree flat-wall cap at N = 16 on 16x8 elements and at N = 8 on
                32x16 (the same node count), one time step;
      isolated: Sec. 3.3, droplet in a 64x64 box, N = 16 on 4x4 elements and N = 4 on
                16x16, La = 3.07, 15, 61.5."""
    from synth import cases
    if kind in ("flat", "curved", "curved-fine"):
        mk = {"flat": cases.paper_flat, "curved": cases.paper_curved,
              "curved-fine": lambda t: cases.paper_curved(t, n_az=64, n_rad=16)}[kind]
        labels = [f"theta {t:g}" for t in (30.0, 60.0, 90.0, 120.0, 150.0)]
        cs = [mk(t) for t in (30.0, 60.0, 90.0, 120.0, 150.0)]
    elif kind == "flat-orders":
        labels = ["theta 60 N 16 16x8", "theta 60 N 8 32x16"]
        cs = [cases.paper_flat(60.0, N=16, nx=16, ny=8), cases.paper_flat(60.0, N=8, nx=32, ny=16)]
    else:
        runs = [(La, N, nel) for N, nel in ((16, 4), (4, 16)) for La in (3.07, 15.0, 61.5)]
        labels = [f"La {La:g} N {N} {nel}x{nel}" for La, N, nel in runs]
        cs = [cases.paper_isolated(La, N, nel) for La, N, nel in runs]
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        if kind in ("isolated", "flat-orders"):
            # one time step for the whole set (the smallest automatic one), so that every
            # run reaches the same T / t_eta at its Laplace number, at both orders
            dts = []
            for c in cs:
                probe = P.Solve(c, stream=stream)
                dts.append(probe.info().dt)
                del probe
            for c in cs:
                c.dt = min(dts)
        solves, meta = [], []
        for c in cs:
            # the library sets tau from the case's viscosity nu at the time step
            s = P.Solve(c, stream=stream)
            s.init_tanh()
            solves.append(s)
            dt = s.info().dt
            c.tau = s.info().tau
            D = 25.6 if kind.startswith("curved") else 32.0
            t_eta = c.rho_l * c.nu * D / c.sigma
            meta.append({"N": c.N, "elements": c.mesh.E, "nu": c.nu, "dt": dt, "tau": c.tau,
                         "t_eta": t_eta, "La": c.sigma * D / (c.rho_l * c.nu ** 2)})
        b = P.Batch(stream)
        for s in solves:
            b.add(s)
        # a run that turns non-finite is reported with the first step it was seen at; the
        # others keep stepping (members of a batch share no data)
        hist, n, t0 = [], 0, time.perf_counter()
        diverged = [None] * len(solves)
        while n < steps and any(d is None for d in diverged):
            b.step(every)
            n += every
            ke = [float(k) for k in b.kinetic_energy()[0]]
            for j, k in enumerate(ke):
                if diverged[j] is None and not math.isfinite(k):
                    diverged[j] = n
            hist.append([n] + [k if math.isfinite(k) else None for k in ke])
            print(f"[paper-{kind}] step {n}: KE_max " + " ".join(f"{k:.2e}" for k in ke),
                  file=sys.stderr, flush=True)
        wall_s = time.perf_counter() - t0
        del b
        angles = []
        if kind != "isolated":
            for s, dv in zip(solves, diverged):
                try:
                    angles.append(s.contact_angle() if dv is None else None)
                except Exception:  # noqa: BLE001 - an unfit interface is reported as null
                    angles.append(None)
    for m in meta:
        m["T_over_t_eta"] = n * m["dt"] / m["t_eta"]
    return {"metric": f"{kind} parasitic currents (KE_max history)", "runs": labels, "params": meta,
            "steps": n, "ke_history": hist, "diverged_at_step": diverged,
            "contact_angle_deg": angles, "wall_s": wall_s,
            "data": "synthetic", "n_gpus": 1, "dtype": "f64"}


def measure_workload(P, torch, name: str, steps: int, warmup: int, profile_steps: int,
                     kernel_reps: int) -> dict:
    """Node-updates/s of one workload (inputs resident, graph-replayed steps between HIP
    events) and the roofline point of its dominant kernel: per-kernel shares of a step from
    HIP events around every launch, then that kernel's launch duration from back-to-back
    launches replayed from one graph on the solve's stream."""
    case = make_case(name)
    m = case.mesh
    Q, d, Ng, Nl = case.lattice, m.dim, m.n_global, m.n_local
    stream = torch.cuda.Stream()  # default priority; capturable (not the null stream)
    with torch.cuda.stream(stream):
        s = P.Solve(case, stream=stream)
        s.init_tanh()
        s.step(warmup)
        torch.cuda.synchronize()
        start, end = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        start.record(stream)
        s.step(steps)
        end.record(stream)
        end.synchronize()
        torch.cuda.synchronize()
        ms = start.elapsed_time(end)
        ke, mass = s.kinetic_energy()
        prof = s.step_profile(profile_steps)
        dom = max(prof, key=lambda k: prof[k][0])
        avg_ms = s.time_kernel(dom, kernel_reps)
        Ni = s.info().n_interior
        del s
    ms_per_step = ms / steps
    tot, nl = prof[dom]
    alg = algorithmic_bytes(dom, Q, d, Ng, Nl, Ni)
    achieved = alg / (avg_ms * 1e-3) / 1e9
    step_gbs = step_model_bytes(Q, d, Ng, Nl) / (ms_per_step * 1e-3) / 1e9
    return {
        "value": Ng * steps / (ms / 1e3),
        "ms_per_step": ms_per_step,
        "config": {"workload": f"{case.name}: " + (case.mesh.name or ""),
                   "lattice": f"D{d}Q{Q}", "N": m.N, "elements": m.E, "n_global": Ng,
                   "n_local": Nl, "n_interior": Ni, "local_node_updates_per_s": Nl * steps / (ms / 1e3),
                   "model_bytes_per_step": step_model_bytes(Q, d, Ng, Nl),
                   "model_GBps": step_gbs,
                   "ke_max_end": ke, "mass_end": mass, "parallelism": "single GPU"},
        "roofline": {"bound": "hbm", "kernel": dom, "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     # the whole step against the step model (model bytes / step time / peak)
                     "step_achieved": step_gbs, "step_frac": step_gbs / HBM_PEAK_GBS,
                     "traffic": traffic_from_profiles(name, dom), "avg_launch_us": avg_ms * 1e3,
                     "launches_timed": kernel_reps,
                     "avg_launch_us_in_step": tot / max(nl, 1) * 1e3,
                     "algorithmic_bytes_per_launch": alg,
                     "kernel_ms_per_step": {k: v[0] / profile_steps for k, v in prof.items()}},
        "fp64": fp64_point(fp64_from_profiles(name), prof, profile_steps, ms_per_step, dom, avg_ms,
                           step_model_bytes(Q, d, Ng, Nl)),
    }


def main():
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=20)
    ap.add_argument("--workload", default="c4",
                    choices=["c1", "c2", "c3", "c4", "c5", "c2xl", "c4q13", "c4n6", "flat16"])
    ap.add_argument("--serve-requests", type=int, default=32)
    ap.add_argument("--serve-max-steps", type=int, default=50000)
    ap.add_argument("--serve-arena-mb", type=int, default=8192,
                    help="server arena: admission stops while the active workspaces fill it")
    ap.add_argument("--no-poisson", action="store_true", help="serving: skip the Poisson-arrival run")
    ap.add_argument("--no-plain", action="store_true", help="serving: skip the one-at-a-time stepper")
    ap.add_argument("--no-serving", action="store_true")
    ap.add_argument("--batch-members", type=int, default=256,
                    help="request-mix solves in the batched-stepping measurement (0: skip)")
    ap.add_argument("--batch-steps", type=int, default=200)
    ap.add_argument("--batch-only", action="store_true",
                    help="only the batched-stepping measurement (one JSON line)")
    ap.add_argument("--profile-steps", type=int, default=100)
    ap.add_argument("--kernel-reps", type=int, default=300)
    ap.add_argument("--cpu-seconds", type=float, default=15.0,
                    help="oracle time budget at one thread (then 6 s at every host thread)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true",
                    help="only the chosen workload: no c2, c2-XL, batch or serving objects")
    ap.add_argument("--paper", choices=["flat", "flat-orders", "curved", "curved-fine", "isolated"],
                    help="only the paper's parasitic-current runs of that test (see paper_runs)")
    ap.add_argument("--paper-steps", type=int, default=4300000)
    ap.add_argument("--paper-every", type=int, default=100000)
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run the byte-counter calibration kernel over MIB MiB")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "the library runs on one GPU: --gpus must be 1 "
                                   "(multi-GPU element partitioning is design-only)"}))
        sys.exit(2)

    import torch

    import paper_2609_00535_amd as P

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU"}))
        sys.exit(1)
    if args.copy_calibration > 0:
        print(json.dumps(copy_calibration(torch, args.copy_calibration)))
        return
    if args.paper:
        print(json.dumps(paper_runs(P, torch, args.paper, args.paper_steps, args.paper_every)))
        return
    if args.batch_only:
        out = batch_bench(P, torch, args.batch_members, args.batch_steps)
        out.update({"metric": "batched FP64 node-updates/s", "value": out["node_updates_per_s"],
                    "unit": "node-updates/s", "n_gpus": 1, "higher_is_better": True, "dtype": "f64",
                    "data": "synthetic", "config": {"workload": f"{args.batch_members} request-mix solves"}})
        print(json.dumps(out))
        return
    if args.workload == "c5":
        out = serving_bench(P, torch, args.serve_requests, args.serve_max_steps,
                            arena_mb=args.serve_arena_mb, poisson=not args.no_poisson,
                            plain=not args.no_plain)
        out.update({"value": out["batched_solves_per_s"], "unit": "solves/s", "n_gpus": 1,
                    "higher_is_better": True, "dtype": "f64", "data": "synthetic",
                    "config": {"workload": f"c5: {args.serve_requests} request-mix solves, each to KE_max < 1e-20 "
                                           f"or {args.serve_max_steps} steps"}})
        print(json.dumps(out))
        return
    r = measure_workload(P, torch, args.workload, args.steps, args.warmup, args.profile_steps,
                         args.kernel_reps)
    out = {
        "metric": "FP64 node-updates/s per step",
        "value": r["value"],
        "unit": "node-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": r["config"],
        "roofline": r["roofline"],
        "fp64": r["fp64"],
    }
    if args.workload == "c4" and not args.no_extras:
        # extra points beside the headline: c2 (a cache-resident, latency-bound 2-D step),
        # c2-XL (a 2-D step whose working set is HBM-resident) and c4 with the D3Q13 lattice
        for key, name, st, wu, ps, kr in (("c2", "c2", 2000, 100, 100, 300),
                                          ("hbm_scale", "c2xl", 100, 10, 3, 20),
                                          ("c4q13", "c4q13", 100, 10, 3, 20)):
            x = measure_workload(P, torch, name, st, wu, ps, kr)
            out[key] = {"workload": x["config"]["workload"], "node_updates_per_s": x["value"],
                        "ms_per_step": x["ms_per_step"], "n_global": x["config"]["n_global"],
                        "model_bytes_per_step": x["config"]["model_bytes_per_step"],
                        "roofline": {k: x["roofline"][k] for k in
                                     ("bound", "kernel", "achieved", "peak", "unit", "frac",
                                      "step_achieved", "step_frac", "traffic", "avg_launch_us",
                                      "algorithmic_bytes_per_launch")},
                        "fp64": x["fp64"]}
        if not args.no_serving:
            if args.batch_members > 0:
                out["batch"] = batch_bench(P, torch, args.batch_members, args.batch_steps)
            out["serving"] = serving_bench(P, torch, args.serve_requests, args.serve_max_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(make_case(args.workload), args.cpu_seconds)
    print(json.dumps(out))


if __name__ == "__main__":
    main()
