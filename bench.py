"""Benchmark of the DCM per-timestep hot path on one MI355X.

Workload: the 2,048,000-particle Lennard-Jones liquid/vapor slab (box 320 x 320 x 60 sigma,
98 % liquid at density 0.8, 2 % vapor, T* = 0.7), cutoffs 2.5..6 sigma from the exponential
cutoff function, interface re-detected every other step, FP64, energy/virial/kinetic thermo
every step. One step = velocity-Verlet kicks and drift, binning (sort-and-segment),
interface detection on even steps, forces.

Prints ONE JSON line: metric, value (atom-steps/s), roofline of the pair-force kernel (FP64
vector ALU), the oracle's CPU baseline on a bounded sample, and a per-stage breakdown.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

FP64_VALU_PEAK_TFLOPS = 78.6     # 256 CU x 4 SIMD x 16 lanes x 2 flop (FMA) x 2.4 GHz
FLOPS_PER_PAIR = 41              # algorithmic FP64 flops per in-range ordered pair
WORKLOAD = "slab2m"
# HBM-side bytes per launch of the FP64 traversal force kernel from FETCH_SIZE/WRITE_SIZE counter runs on the slab's
# lattice start (--forces-only), scaled by a plain 1 GiB copy (profiles/KForces_slab2m_traffic.md).
# Valid only for the kernel source it was taken on: reported as null once csrc/force.hip no longer
# hashes to this value.
FORCE_TRAFFIC_BYTES = 3.13e9
FORCE_TRAFFIC_SRC = "89513ad104e69f27"


def force_traffic():
    import hashlib
    path = os.path.join(ROOT, "paper_1502_03234_amd", "csrc", "force.hip")
    with open(path, "rb") as f:
        h = hashlib.sha256(f.read()).hexdigest()[:16]
    return FORCE_TRAFFIC_BYTES if h == FORCE_TRAFFIC_SRC else None


def stage_bandwidth(breakdown: dict, n: int, G: int, detect_every: int) -> dict:
    """Achieved bandwidth of the HBM-bound stages: algorithmic bytes per step / stage time.
    Per particle: kick/drift/key 144 B (read x, v, F; write x, v, key and the rank in its cell,
    which the counting sort's count takes here); binning 144 B (scatter: key, rank and cell
    start read, key and source slot written, 20 B; in-cell order 4 B; gather 120 B) plus 16 B
    per box (its two storage cells' counts read and starts written; clearing the occupied
    cells' counts is not counted) plus, per box and detection, the box-count image the cell
    scan writes (4 B). Per box and detection: smoothing 8 B (one fused [1,2,1]^3 pass),
    two-means 4 B (histogram read), labels and components 66 B (threshold 6 B, two component passes of about 30 B). Per particle
    and detection: cutoffs 96 B (eight 8-byte box values, the 32-byte position record read).
    Detection stages count once per detect_every steps. The distance solve's floor is reading
    the labels and writing the distances once, 9 B per box and detection; it runs far above that
    floor (its relaxation passes are bound by LDS arithmetic and pass latency), which the
    achieved figure shows."""
    per_det = 1.0 / detect_every if detect_every > 0 else 0.0
    bytes_per_step = {
        "kick_drift_key": 144.0 * n,
        "sort": 144.0 * n + 16.0 * G + 4.0 * G * per_det,
        "smooth": 8.0 * G * per_det,
        "two_means": 4.0 * G * per_det,
        "segment": 66.0 * G * per_det,
        "distance": 9.0 * G * per_det,
        "cutoffs": 96.0 * n * per_det,
    }
    out = {}
    for k, b in bytes_per_step.items():
        ms = breakdown.get(k, 0.0)
        if ms > 0 and b > 0:
            gbs = b / (ms * 1e-3) / 1e9
            out[k] = {"bytes_per_step": b, "GB_per_s": round(gbs, 1), "frac_of_hbm": round(gbs / 8000.0, 3)}
    return out


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def cpu_baseline(state, sample: int, seed: int = 12345, total_pairs: float | None = None):
    """Time the CPU oracle on a bounded sample of the same workload: one interface detection
    on the full state (charged at 1/2 per step: detection every other step), forces for a
    seeded random sample of particles, and one full velocity-Verlet position/velocity update.
    The sample's force time is scaled to all particles by their number; with total_pairs (the
    whole system's in-range pair count) it is also scaled by pairs, and the two estimates are
    reported side by side (their spread bounds the sampling error of the extrapolation)."""
    import numpy as np
    import oracle as O

    p = O.params(state.box)
    x = O.wrap(p, state.x)
    t0 = time.perf_counter()
    det = O.detect(p, x)
    t_det = time.perf_counter() - t0
    idx = np.sort(np.random.default_rng(seed).choice(state.n, sample, replace=False))
    t0 = time.perf_counter()
    fr = O.forces(p, x, det.rc, subset=idx)
    t_sample = time.perf_counter() - t0
    t_f = t_sample / sample * state.n
    sample_pairs = float(fr.pairs.sum())
    v = state.v.copy()
    f = np.zeros_like(v)
    t0 = time.perf_counter()
    v += 0.0025 * f
    x2 = x + 0.005 * v
    O.wrap(p, x2)
    v += 0.0025 * f
    t_int = time.perf_counter() - t0
    per_step = t_f + 0.5 * t_det + t_int
    out = dict(value=state.n / per_step, unit="atom-steps/s", cores=1, kind="oracle",
               sample=(f"slab2m, the state the GPU timing starts from: detection on all {state.n} particles (x1/2 per step), forces "
                       f"for {sample} seeded random particles scaled to {state.n}, one full "
                       f"integration update; {per_step:.1f} s per step"),
               seconds=dict(detect=t_det, forces_sample=t_sample, forces_scaled=t_f, integrate=t_int))
    if total_pairs:
        t_fp = t_sample * total_pairs / sample_pairs
        per_step_p = t_fp + 0.5 * t_det + t_int
        out["by_pairs"] = dict(value=state.n / per_step_p, sample_pairs_per_particle=sample_pairs / sample,
                               pairs_per_particle=total_pairs / state.n,
                               rel_diff=per_step_p / per_step - 1.0)
    return out


def under_profiler() -> bool:
    """True when a profiler tool is loaded into this process (rocprofv3 announces itself through
    ROCPROF_* variables). Child processes would inherit the tool."""
    return any(k.startswith("ROCPROF") for k in os.environ)


def host_cpu() -> dict:
    """CPU model, logical CPUs of the host and CPUs this process may run on."""
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    try:
        usable = len(os.sched_getaffinity(0))
    except (AttributeError, OSError):
        usable = os.cpu_count() or 1
    return {"model": model, "nproc": os.cpu_count() or 1, "usable": usable}


def save_state(state, x, v):
    """Writes a state (positions and velocities in caller order) for the oracle workers."""
    import tempfile
    import numpy as np
    fd, path = tempfile.mkstemp(suffix=".npz", dir="/dev/shm" if os.path.isdir("/dev/shm") else None)
    os.close(fd)
    np.savez(path, x=x, v=v, box=np.array(state.box))
    return path


def cpu_workers_start(sample: int, procs: int):
    """Starts `procs` oracle processes (bench.py --cpu-worker) before this process touches the
    GPU, so that no process holding a GPU context forks. Each waits on its stdin for the path of
    the state to run on; cpu_workers_collect sends it once the GPU timing is over, so that they
    do not compete with it for host cores and work on the state the GPU timing measured."""
    import subprocess
    workers = []
    for k in range(procs):
        workers.append(subprocess.Popen(
            [sys.executable, os.path.abspath(__file__), "--cpu-worker", "stdin", "--cpu-sample", str(sample),
             "--cpu-seed", str(12345 + k)],
            stdin=subprocess.PIPE, stdout=subprocess.PIPE, stderr=subprocess.DEVNULL, text=True))
    return {"workers": workers}


def cpu_workers_collect(handle, path: str, timeout_s: float = 600.0):
    """Releases the workers at once on the state in `path` and sums their throughput: the
    host's aggregate figure."""
    ws = handle["workers"]
    try:
        for w in ws:
            w.stdin.write(path + "\n")
            w.stdin.flush()
        vals = []
        for w in ws:
            out, _ = w.communicate(timeout=timeout_s)
            vals.append(float(json.loads(out.strip().splitlines()[-1])["value"]))
    finally:
        for w in ws:
            if w.poll() is None:
                w.kill()
                w.wait()
    return dict(value=float(sum(vals)), unit="atom-steps/s", cores=len(ws), kind="oracle",
                sample=f"{len(ws)} independent oracle processes at once, each on the single-core sample")


def cpu_worker_main(sample: int, seed: int):
    """One oracle copy of the bounded sample, started by cpu_workers_start; it never touches
    the GPU. Waits for the path of the state on its stdin, runs, prints one JSON line."""
    import numpy as np
    from types import SimpleNamespace
    path = sys.stdin.readline().strip()
    if not path:
        return
    d = np.load(path)
    st = SimpleNamespace(x=d["x"], v=d["v"], box=tuple(float(b) for b in d["box"]), n=d["x"].shape[1])
    print(json.dumps({"value": cpu_baseline(st, sample, seed)["value"]}), flush=True)


def _fp64_forces_of(p, x, v, rc, k):
    """Forces of the FP64 form on a given state and cutoffs (a system that never re-detects, so
    the cutoffs are used as given). The FP64 form's agreement with the oracle is what the parity
    tests establish; here it is the reference of the FP32 form."""
    from paper_1502_03234_amd import dcm
    q = dcm.Params.from_buffer_copy(p)
    q.precision, q.detect_every = dcm.DCM_FP64, 0
    r = dcm.System(q, x, v, rc=rc, step=k)
    f = r.forces(per_atom=False, thermo=False)["f"]
    r.close()
    return f


def _form_error(f, ref):
    """Per-atom |dF_i| / max(|F_i|, F_rms) over all particles: max and rms."""
    import torch
    frms = torch.sqrt(torch.mean(torch.sum(ref ** 2, dim=0)))
    e = torch.linalg.norm(f - ref, dim=0) / torch.clamp(torch.linalg.norm(ref, dim=0), min=frms)
    return float(e.max()), float(torch.sqrt(torch.mean(e ** 2)))


def precision_study(nsteps: int):
    """Both forms on the 256,000-particle slab with shifted pair energies: total-energy drift
    per particle over nsteps, and the FP32 form's per-atom force error |dF_i| / max(|F_i|,
    F_rms) against the FP64 form on every particle of the FP32 form's own state and cutoffs
    (checkpoints at 0, nsteps/2 and nsteps)."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("slab256k")
    out = {"study": "precision", "workload": "LJ slab 256,000 particles, box 112x112x60, shifted pair "
           "energies, detect every 2nd step", "steps": nsteps, "forms": {}}
    for name, prec in (("f64", dcm.DCM_FP64), ("f32c", dcm.DCM_FP32C)):
        p = dcm.params(st.box, precision=prec, energy_shift=1)
        s = dcm.System(p, st.x, st.v)
        errs, energies = [], []
        half = nsteps // 2
        for leg in (0, half, nsteps - half):
            if leg:
                th = dcm.thermo_records(s.step(leg))
                energies += [r["ke"] + r["pe"] for r in th]
            fo = s.forces(per_atom=False, thermo=(not energies))
            if not energies:
                t0 = dcm.thermo_records(fo["thermo"])[0]
                energies.append(t0["ke"] + t0["pe"])
            if prec == dcm.DCM_FP32C:
                x, v, rc, k = s.state()
                emax, erms = _form_error(fo["f"], _fp64_forces_of(p, x, v, rc, k))
                errs.append({"step": k, "max": emax, "rms": erms})
                log(f"{name} step {k}: force error vs the FP64 form, max {emax:.3e}")
        s.check()
        en = np.array(energies) / st.n
        out["forms"][name] = {"energy_per_particle_start": float(en[0]),
                              "drift_per_particle": float(en[-1] - en[0]),
                              "max_excursion_per_particle": float(np.max(np.abs(en - en[0]))),
                              "force_error_vs_f64": errs}
        s.close()
    print(json.dumps(out), flush=True)


def droplet_study(nsteps: int):
    """Non-planar interface: the 1,000,000-particle droplet (radius 66.83, box 166^3, vapor at
    0.01), both forms, shifted pair energies, detection every 2nd step. Reports the detected
    segmentation against the analytic sphere (boxes whose centre lies more than 3 sigma from the
    sphere must carry its label; the radius of a sphere with the detected liquid volume), the
    FP32 form's per-atom force error against the FP64 form on every particle of its own state
    at steps 0 and nsteps, the total-energy drift per particle, and atom-steps/s."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("droplet1m")
    R, c = st.meta["radius"], st.meta["centre"]
    out = {"study": "droplet", "workload": f"LJ droplet {st.n_liquid} particles (R = {R:.3f}) + "
           f"{st.n_vapor} vapor, box 166^3, shifted pair energies, detect every 2nd step",
           "n_particles": st.n, "steps": nsteps, "forms": {}}
    for name, prec in (("f64", dcm.DCM_FP64), ("f32c", dcm.DCM_FP32C)):
        p = dcm.params(st.box, precision=prec, energy_shift=1)
        s = dcm.System(p, st.x, st.v)
        det = s.detect()
        dims = dcm.dcm_grid_dims(p)
        lab = det["label"].cpu().numpy().reshape(dims[2], dims[1], dims[0])
        h = [st.box[k] / dims[k] for k in range(3)]
        zc, yc, xc = np.meshgrid(*[(np.arange(dims[k]) + 0.5) * h[k] for k in (2, 1, 0)], indexing="ij")
        r = np.sqrt((xc - c) ** 2 + (yc - c) ** 2 + (zc - c) ** 2)
        far = np.abs(r - R) > 3.0
        wrong = lab != (r > R)
        seg = {"far_boxes": int(far.sum()), "far_label_errors": int((wrong & far).sum()),
               "max_error_distance_from_sphere": float(np.abs(r - R)[wrong].max()) if wrong.any() else 0.0,
               "radius_from_liquid_volume": float((3.0 * np.prod(h) * (lab == 0).sum() / (4.0 * np.pi)) ** (1 / 3)),
               "radius_analytic": float(R)}
        errs, energies = [], []
        ms = None
        for leg in (0, nsteps):
            if leg:
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                th = dcm.thermo_records(s.step(leg))
                torch.cuda.synchronize()
                ms = (time.perf_counter() - t0) * 1e3 / leg
                energies += [q["ke"] + q["pe"] for q in th]
            fo = s.forces(per_atom=False, thermo=(not energies))
            if not energies:
                energies.append(sum(dcm.thermo_records(fo["thermo"])[0][k] for k in ("ke", "pe")))
            if prec == dcm.DCM_FP32C:
                x, v, rc, k = s.state()
                emax, erms = _form_error(fo["f"], _fp64_forces_of(p, x, v, rc, k))
                errs.append({"step": k, "max": emax, "rms": erms})
                log(f"droplet {name} step {k}: force error vs the FP64 form, max {emax:.3e}")
        s.check()
        en = np.array(energies) / st.n
        out["forms"][name] = {"segmentation": seg, "force_error_vs_f64": errs,
                              "drift_per_particle": float(en[-1] - en[0]),
                              "max_excursion_per_particle": float(np.max(np.abs(en - en[0]))),
                              "ms_per_step": ms, "atom_steps_per_s": st.n * 1e3 / ms}
        s.close()
    print(json.dumps(out), flush=True)


def serving_study(nseeds: int, nsys: int = 64, nsteps: int = 100, load: float = 0.8,
                  droplets: bool = False, emit: bool = True):
    """Serving form against one-system-at-a-time solves on the same Poisson traces.

    Systems: 64 slabs (with `droplets`, every 4th system a droplet of the same size in vapor),
    N log-uniform on [4,000, 200,000], T* uniform on [0.65, 0.85], 100 steps each. Sequential: every request is solved alone (H2D copy, create, 100 steps, D2H copy);
    its wall-clock service time is measured once and the FIFO timeline of each trace follows
    from the arrival times (exact for a single FIFO server). Capacity = requests / sum of
    service times; arrivals are Poisson at load x capacity. Server: the same requests are
    submitted at their arrival times to a dcm_server whose HBM budget is a quarter of the
    trace's total footprint, so admission queues. Latency = completion - arrival."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    trace = synth.serving_trace(1, nsys)
    systems = [synth.serving_droplet(j, n, t) if droplets and j % 4 == 3 else synth.serving_system(j, n, t)
               for j, (n, t) in enumerate(trace)]
    params = [dcm.params(s.box) for s in systems]
    sizes = np.array([s.n for s in systems])
    log(f"serving: {nsys} systems, {sizes.sum()} particles, sizes {sizes.min()}..{sizes.max()}")
    # sequential service times, after one untimed solve of the first system (library and
    # allocator warm-up would otherwise be charged to it)
    warm = dcm.System(params[0], torch.from_numpy(systems[0].x).cuda(), torch.from_numpy(systems[0].v).cuda())
    warm.step(nsteps, thermo=True)
    torch.cuda.synchronize()
    warm.close()
    svc = np.zeros(nsys)
    for j, (s, p) in enumerate(zip(systems, params)):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        x = torch.from_numpy(s.x).cuda()
        v = torch.from_numpy(s.v).cuda()
        sysm = dcm.System(p, x, v)
        sysm.step(nsteps, thermo=True)
        xo, vo, rc, k = sysm.state()
        xo.cpu(), vo.cpu()
        torch.cuda.synchronize()
        svc[j] = time.perf_counter() - t0
        sysm.close()
    cap = nsys / svc.sum()
    rate = load * cap
    foot = [dcm.dcm_workspace_bytes(p, s.n) + 48 * s.n + 4096 for s, p in zip(systems, params)]
    budget = max(int(0.25 * sum(foot)), max(foot) + 4096)
    pool = dcm.workspace(int(1.25 * budget))
    seq_lat, srv_lat, seq_tp, srv_tp, srv_stats = [], [], [], [], []
    atom_steps = float(sizes.sum()) * nsteps
    for seed in range(1, nseeds + 1):
        order = np.random.default_rng(seed).permutation(nsys)
        arr = synth.poisson_arrivals(seed, nsys, rate)
        # sequential FIFO timeline
        t, lat = 0.0, []
        for a, j in zip(arr, order):
            t = max(t, a) + svc[j]
            lat.append(t - a)
        seq_lat += lat
        seq_tp.append(atom_steps / (t - arr[0]))
        # server, real time
        sv = dcm.dcm_server_create(budget, pool)
        t0 = time.perf_counter()
        tickets, done = {}, {}
        nxt = 0
        while len(done) < nsys:
            now = time.perf_counter() - t0
            while nxt < nsys and arr[nxt] <= now:
                j = order[nxt]
                tickets[dcm.dcm_submit(sv, params[j], systems[j].x, systems[j].v, nsteps)] = (j, arr[nxt])
                nxt += 1
            for tk, (j, a) in list(tickets.items()):
                st = dcm.dcm_poll(sv, tk, systems[j].n)[0]
                if st == dcm.DCM_OK:
                    done[tk] = (time.perf_counter() - t0) - a
                    del tickets[tk]
            time.sleep(0.0005)
        last = time.perf_counter() - t0
        stats = dcm.dcm_server_query(sv)
        dcm.dcm_server_destroy(sv)
        srv_lat += list(done.values())
        srv_tp.append(atom_steps / (last - arr[0]))
        log(f"seed {seed}: server p50 {np.percentile(list(done.values()), 50):.3f}s, "
            f"batches {stats['batches']}, groupings {stats['groupings']} "
            f"({stats['grouping_ms']:.1f} ms), grouped/eager periods {stats['grouped_steps']}/"
            f"{stats['eager_steps']}, sequential p50 {np.percentile(lat, 50):.3f}s")
        srv_stats.append(stats)
    # saturated: every request arrives at t = 0; makespan against the sum of service times
    sv = dcm.dcm_server_create(budget, pool)
    t0 = time.perf_counter()
    tickets = {dcm.dcm_submit(sv, params[j], systems[j].x, systems[j].v, nsteps): j
               for j in range(nsys)}
    while tickets:
        for tk, j in list(tickets.items()):
            if dcm.dcm_poll(sv, tk, systems[j].n)[0] == dcm.DCM_OK:
                del tickets[tk]
        time.sleep(0.0005)
    makespan = time.perf_counter() - t0
    sat_stats = dcm.dcm_server_query(sv)
    dcm.dcm_server_destroy(sv)
    log(f"saturated: server makespan {makespan:.3f}s, sequential {svc.sum():.3f}s, batches "
        f"{sat_stats['batches']}, groupings {sat_stats['groupings']} ({sat_stats['grouping_ms']:.1f} ms)")
    out = {"study": "serving", "mix": "slabs and droplets (every 4th)" if droplets else "slabs", "systems": nsys, "steps_each": nsteps, "seeds": nseeds,
           "particles_total": int(sizes.sum()), "load": load, "arrival_rate_per_s": rate,
           "hbm_budget_bytes": budget, "sequential_capacity_req_per_s": cap,
           "server": {"throughput_atom_steps_per_s": float(np.mean(srv_tp)),
                      "p50_latency_s": float(np.percentile(srv_lat, 50)),
                      "p99_latency_s": float(np.percentile(srv_lat, 99))},
           "sequential": {"throughput_atom_steps_per_s": float(np.mean(seq_tp)),
                          "p50_latency_s": float(np.percentile(seq_lat, 50)),
                          "p99_latency_s": float(np.percentile(seq_lat, 99))},
           "saturated": {"server_atom_steps_per_s": atom_steps / makespan,
                         "sequential_atom_steps_per_s": atom_steps / float(svc.sum()),
                         "makespan_s": makespan, "server_stats": sat_stats},
           "server_stats_per_seed": srv_stats,
           "samples": len(srv_lat)}
    if emit:
        print(json.dumps(out), flush=True)
    return out


# Total energy per particle printed by the thesis (Section 6, Table 1) for its 16,000-particle
# slab after 100,000 NVT steps at T* = 0.7, dt = 0.005; the quoted standard deviations are
# 0.013-0.017. Keys: (r_c^min, r_c^max); equal values are the static cutoff.
TABLE1_ENERGY = {(3.0, 3.0): -4.415, (5.0, 5.0): -4.772, (7.0, 7.0): -4.830,
                 (3.0, 5.0): -4.557, (3.0, 7.0): -4.636, (3.0, 8.0): -4.660,
                 (4.5, 9.5): -4.805}


def nvt_study(equil: int, sample: int, configs=None, chunk: int = 1000, tdamp: float = 0.5,
              save_dir: str | None = None, detect_kw: dict | None = None):
    """Table 1 and Figure 37 observables. The thesis's geometry (16,000 particles in a 22 x 22 x
    44 block centred in 22 x 22 x 88), Nose-Hoover at T* = 0.7, dt = 0.005, unshifted pair
    energies, detection every 2nd step; one system per Table 1 cutoff configuration, all
    stepped concurrently on streams of their own. After `equil` steps, `sample` steps give:
    total energy per particle (block averages over `chunk` steps, standard error of the block
    means), the density profile along z about the slab's centre (liquid |dz| < 10, vapor
    |dz| > 30), and the surface tension Lz/2 <P_zz - (P_xx + P_yy)/2> from the virial (the
    kinetic part of the pressure tensor is isotropic on average and drops out). Then each
    configuration alone: ms per step. With save_dir, each final state (x, v, r_c in caller order,
    the thermostat's xi and eta) is written there as an .npz file."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("thesis16k")
    Lx, Ly, Lz = st.box
    V = Lx * Ly * Lz
    edges = np.arange(-Lz / 2, Lz / 2 + 1e-9, 1.0)
    systems = []
    for q, ((rmin, rmax), ref) in enumerate(TABLE1_ENERGY.items()):
        if configs is not None and q not in configs:
            continue
        p = dcm.params(st.box, rc_min=rmin, rc_max=rmax, thermostat=dcm.DCM_NOSE_HOOVER,
                       temperature=0.7, tdamp=tdamp, **(detect_kw or {}))
        stream = torch.cuda.Stream()
        s = dcm.System(p, st.x, st.v, stream=stream)
        systems.append(dict(name=("static %.1f" % rmax) if rmin == rmax else "DCM %.1f/%.1f" % (rmin, rmax),
                            rc=(rmin, rmax), ref=ref, s=s, stream=stream,
                            th=torch.empty(chunk * dcm.THERMO_DOUBLES, dtype=torch.float64, device="cuda"),
                            x=torch.empty((3, st.n), dtype=torch.float64, device="cuda"),
                            E=[], gamma=[], T=[], hist=np.zeros(len(edges) - 1), frames=0))
    total = equil + sample
    t0 = time.perf_counter()
    done = 0
    while done < total:
        for c in systems:
            dcm.dcm_step(c["s"].h, chunk, c["stream"], c["th"])
        torch.cuda.synchronize()
        done += chunk
        if done > equil:
            for c in systems:
                rec = dcm.thermo_records(c["th"])
                e = np.array([r["ke"] + r["pe"] for r in rec]) / st.n
                w = np.array([r["virial"] for r in rec])
                c["E"].append(e.mean())
                c["gamma"].append(np.mean(0.5 * Lz * (w[:, 2] - 0.5 * (w[:, 0] + w[:, 1])) / V))
                c["T"].append(np.mean([2.0 * r["ke"] / (3 * st.n - 3) for r in rec]))
                dcm.dcm_get_state(c["s"].h, c["stream"], x=c["x"])
            torch.cuda.synchronize()
            for c in systems:
                z = c["x"][2].cpu().numpy()
                th = 2 * np.pi * z / Lz
                zc = math.atan2(np.sin(th).mean(), np.cos(th).mean()) * Lz / (2 * np.pi)
                dz = np.mod(z - zc + Lz / 2, Lz) - Lz / 2
                c["hist"] += np.histogram(dz, bins=edges)[0]
                c["frames"] += 1
        if done % (10 * chunk) == 0 or done == total:
            log(f"nvt study: {done}/{total} steps of {len(systems)} systems, "
                f"{time.perf_counter() - t0:.1f} s")
    rows = []
    mid = 0.5 * (edges[1:] + edges[:-1])
    for c in systems:
        c["s"].check()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        dcm.dcm_step(c["s"].h, 500, c["stream"], None)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 2.0
        if save_dir:
            xs, vs, rcs, k = c["s"].state()
            xi, eta = c["s"].thermostat()
            os.makedirs(save_dir, exist_ok=True)
            np.savez(os.path.join(save_dir, "thesis16k_nvt_%g_%g.npz" % c["rc"]), x=xs.cpu().numpy(),
                     v=vs.cpu().numpy(), rc=rcs.cpu().numpy(), step=k, xi=xi, eta=eta)
        E = np.array(c["E"])
        g = np.array(c["gamma"])
        rho = c["hist"] / (Lx * Ly * 1.0 * max(c["frames"], 1))
        se = lambda a: float(a.std(ddof=1) / math.sqrt(len(a))) if len(a) > 1 else None
        rows.append({"config": c["name"], "rc_min": c["rc"][0], "rc_max": c["rc"][1],
                     "E_per_particle": float(E.mean()), "E_stderr": se(E),
                     "E_table1": c["ref"], "E_minus_table1": float(E.mean() - c["ref"]),
                     "T_mean": float(np.mean(c["T"])),
                     "rho_liquid": float(rho[np.abs(mid) < 10].mean()),
                     "rho_vapor": float(rho[np.abs(mid) > 30].mean()),
                     "gamma": float(g.mean()), "gamma_stderr": se(g), "ms_per_step": ms,
                     "profile": [round(float(r), 4) for r in rho]})
        c["s"].close()
    out = {"study": "nvt_table1", "workload": "16,000 LJ particles, 22 x 22 x 44 block in a 22 x 22 x 88 "
           "box (thesis Section 6), Nose-Hoover T* = 0.7 tau = %g, dt = 0.005, unshifted energies, "
           "detect every 2nd step" % tdamp, "equil_steps": equil, "sample_steps": sample,
           "block_steps": chunk, "detection": detect_kw or {}, "wall_s": time.perf_counter() - t0,
           "rows": rows}
    print(json.dumps(out), flush=True)


def accuracy_study(equil: int, R: float = 20.0, time_steps: int = 200, detect_kw: dict | None = None):
    """Force accuracy of the cutoff method (Section 6.1.1, Eq. 20; Figures 34-36 analogues) on
    the thesis's 16,000-particle slab. The lattice start is equilibrated for `equil` NVT steps
    (Nose-Hoover, T* = 0.7, static cutoff 5.0); on that one state, the exact forces are the
    full Lennard-Jones image sum within R (dcm_exact_forces), and every (r_c^min, r_c^max,
    cutoff shape) configuration of the grid below is evaluated on the same positions: interface
    detection, cutoffs, Alg. 3.2 forces. Errors per configuration:
      rel_rms = sqrt(sum_i |F_i - F_i^ex|^2 / sum_i |F_i^ex|^2)   (Eq. 20 with the vector
                quotient read as a ratio of mean squares, well conditioned where F^ex ~ 0);
      eq20_mag = sqrt(mean_i (|F_i - F_i^ex| / |F_i^ex|)^2)       (Eq. 20 per particle with
                magnitudes; dominated by particles whose exact force is small);
    and the mean signed error of F_z in 2-sigma slices about the slab's centre (Figure 35).
    ms/step is timed over `time_steps` NVE steps from that state for each configuration, and for
    each accuracy threshold the cheapest configuration meeting it is listed (Figure 36's
    arrows), by pairs per particle and by step time."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("thesis16k")
    Lz = st.box[2]
    t0 = time.perf_counter()
    p_eq = dcm.params(st.box, rc_min=5.0, rc_max=5.0, thermostat=dcm.DCM_NOSE_HOOVER,
                      temperature=0.7, tdamp=0.5)
    s = dcm.System(p_eq, st.x, st.v)
    chunk = 10000
    for k in range(0, equil, chunk):
        s.step(min(chunk, equil - k), thermo=False)
        torch.cuda.synchronize()
        log(f"accuracy study: equilibrated {min(k + chunk, equil)}/{equil} steps")
    s.check()
    x, v, _, _ = s.state()
    fex = s.exact_forces(R)
    torch.cuda.synchronize()
    s.close()
    fex_h = fex.cpu().numpy()
    xw = x.cpu().numpy()
    th = 2 * np.pi * xw[2] / Lz
    zc = math.atan2(np.sin(th).mean(), np.cos(th).mean()) * Lz / (2 * np.pi)
    dz = np.mod(xw[2] - zc + Lz / 2, Lz) - Lz / 2
    edges = np.arange(-Lz / 2, Lz / 2 + 1e-9, 2.0)
    sl = np.clip(np.digitize(dz, edges) - 1, 0, len(edges) - 2)
    nslab = np.bincount(sl, minlength=len(edges) - 1)
    fex_rms = float(np.sqrt(np.mean(np.sum(fex_h ** 2, axis=0))))
    log(f"accuracy study: exact forces (R = {R}), F_rms = {fex_rms:.4f}")

    grid = []
    for rmin in (2.5, 3.0, 3.5, 4.0, 4.5, 5.0, 6.0, 7.0):
        for rmax in (3.0, 4.0, 5.0, 5.5, 6.0, 7.0, 8.0, 9.0, 10.0):
            if rmax < rmin:
                continue
            shapes = (dcm.DCM_CUTOFF_EXP,) if rmin == rmax else (dcm.DCM_CUTOFF_EXP, dcm.DCM_CUTOFF_LINEAR)
            for shape in shapes:
                grid.append((rmin, rmax, shape))
    rows = []
    for rmin, rmax, shape in grid:
        try:
            p = dcm.params(st.box, rc_min=rmin, rc_max=rmax, cutoff_shape=shape, **(detect_kw or {}))
            dcm.dcm_workspace_bytes(p, st.n)
        except dcm.DcmError as exc:       # e.g. a stencil wider than the box at coarse bins
            log(f"accuracy study: skipping {rmin}/{rmax}: {exc}")
            continue
        s = dcm.System(p, x, v)
        fo = s.forces(per_atom=False, thermo=True)
        f = fo["f"]
        _, _, rc, _ = s.state()
        torch.cuda.synchronize()
        pairs = dcm.thermo_records(fo["thermo"])[0]["pairs"]
        d = f.cpu().numpy() - fex_h
        dn = np.linalg.norm(d, axis=0)
        en = np.linalg.norm(fex_h, axis=0)
        ok = en > 0
        prof = np.bincount(sl, weights=d[2], minlength=len(edges) - 1) / np.maximum(nslab, 1)
        s.step(10, thermo=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        s.step(time_steps, thermo=False)
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / time_steps
        s.check()
        s.close()
        name = ("static %.1f" % rmin) if rmin == rmax else \
            "DCM %.1f/%.1f %s" % (rmin, rmax, "exp" if shape == dcm.DCM_CUTOFF_EXP else "linear")
        rows.append({"config": name, "rc_min": rmin, "rc_max": rmax,
                     "shape": "exp" if shape == dcm.DCM_CUTOFF_EXP else "linear",
                     "rel_rms": float(np.sqrt(np.sum(dn ** 2) / np.sum(en ** 2))),
                     "eq20_mag": float(np.sqrt(np.mean((dn[ok] / en[ok]) ** 2))),
                     "max_abs": float(dn.max()), "mean_rc": float(rc.mean()),
                     "pairs_per_particle": pairs / st.n,
                     "ms_per_step": ms, "dFz_profile": [round(float(q), 6) for q in prof]})
        log(f"accuracy study: {name}: rel_rms {rows[-1]['rel_rms']:.5f}, {ms:.3f} ms/step")
    # cheapest configuration meeting each threshold, by pairs per particle (the work of
    # Alg. 3.2, which sets the step time of large systems) and by the measured step time (a
    # 16,000-particle step is mostly launch latency on one GPU)
    best = []
    for thr in (0.005, 0.003, 0.002, 0.0015, 0.00133, 0.001, 0.0007, 0.0005, 0.0003, 0.0002, 0.0001):
        cand = [r for r in rows if r["shape"] == "exp" and r["rel_rms"] <= thr]
        if cand:
            b = min(cand, key=lambda r: r["pairs_per_particle"])
            t = min(cand, key=lambda r: r["ms_per_step"])
            best.append({"threshold": thr, "by_pairs": b["config"], "rel_rms": b["rel_rms"],
                         "pairs_per_particle": b["pairs_per_particle"], "by_time": t["config"],
                         "ms_per_step": t["ms_per_step"]})
    out = {"study": "accuracy", "workload": "thesis 16,000-particle slab (22 x 22 x 44 block in 22 x 22 "
           f"x 88), NVT-equilibrated {equil} steps at static r_c = 5.0, T* = 0.7", "R_exact": R,
           "F_rms_exact": fex_rms, "slices_2sigma_from": float(edges[0]), "rows": rows,
           "fastest_meeting_threshold": best, "detection": detect_kw or {},
           "wall_s": time.perf_counter() - t0}
    print(json.dumps(out), flush=True)


def oracle_study(steps16k: int = 100, steps256k: int = 5):
    """The single-threaded CPU oracle against the HIP path on the smaller configurations, whole
    runs rather than samples: the 16,000-particle slab for `steps16k` steps and the
    256,000-particle slab for `steps256k` steps (each from the generated state, detection every
    2nd step, FP64, NVE). Per configuration: seconds per step on each side and the ratio."""
    import numpy as np
    import torch
    import oracle as O
    from paper_1502_03234_amd import dcm, synth

    rows = []
    for name, k in (("slab16k", steps16k), ("slab256k", steps256k)):
        st = synth.named(name)
        p = dcm.params(st.box)
        s = dcm.System(p, st.x, st.v)
        s.step(2, thermo=False)
        torch.cuda.synchronize()
        s.close()
        s = dcm.System(p, st.x, st.v)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s.step(k, thermo=False)
        torch.cuda.synchronize()
        gpu = (time.perf_counter() - t0) / k
        s.check()
        s.close()
        po = O.params(st.box)
        t0 = time.perf_counter()
        rs = O.prepare(po, st.x, st.v)
        t_prep = time.perf_counter() - t0
        t0 = time.perf_counter()
        O.run(po, rs, k)
        cpu = (time.perf_counter() - t0) / k
        row = {"config": name, "n": st.n, "steps": k, "gpu_s_per_step": gpu, "oracle_s_per_step": cpu,
               "oracle_setup_s": t_prep, "ratio": cpu / gpu,
               "gpu_atom_steps_per_s": st.n / gpu, "oracle_atom_steps_per_s": st.n / cpu}
        if name == "slab256k":
            # the headline's sampled estimate (the same 60,000 / 2,048,000 share of particles)
            # against this whole run, on the same host: its extrapolation error
            sample = int(round(st.n * 60000 / 2048000))
            cb = cpu_baseline(st, sample)
            est = st.n / cb["value"]
            row["sampled_estimate"] = {"sample": sample, "s_per_step": est, "rel_err_vs_whole_run": est / cpu - 1.0}
            log(f"oracle study: sampled estimate {est:.3f} s/step against the whole run's {cpu:.3f} "
                f"({100 * (est / cpu - 1.0):+.1f} %)")
        rows.append(row)
        log(f"oracle study: {name}: GPU {gpu * 1e3:.3f} ms/step, oracle {cpu:.3f} s/step, ratio {cpu / gpu:.0f}")
    out = {"study": "oracle_timing", "oracle": "dcm_oracle.c, gcc -O2, one thread", "cores": 1,
           "host_cpu": _host_cpu(), "rows": rows}
    print(json.dumps(out), flush=True)


def _host_cpu() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def profile_study(nsteps: int = 100):
    """Cutoff profile over the density profile (Figure 33 analogue): the 16,000-particle slab
    (28 x 28 x 60) after `nsteps` NVE steps, for the default cutoffs (2.5 / 6.0) and the
    thesis's Figure 33 pair (4.0 / 7.0). Per 1-sigma slice of z: number density, and the mean,
    minimum and maximum r_c of the particles in the slice."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("slab16k")
    Lx, Ly, Lz = st.box
    edges = np.arange(0.0, Lz + 1e-9, 1.0)
    out = {"study": "cutoff_profile", "workload": f"LJ slab 16,000 particles, box 28x28x60, {nsteps} NVE "
           "steps, detect every 2nd step", "z_slices": [float(e) for e in edges[:-1]], "configs": []}
    for rmin, rmax in ((2.5, 6.0), (4.0, 7.0)):
        s = dcm.System(dcm.params(st.box, rc_min=rmin, rc_max=rmax), st.x, st.v)
        s.step(nsteps, thermo=False)
        x, _, rc, k = s.state()
        torch.cuda.synchronize()
        s.check()
        s.close()
        z = x[2].cpu().numpy()
        r = rc.cpu().numpy()
        sl = np.clip(np.digitize(z, edges) - 1, 0, len(edges) - 2)
        cnt = np.bincount(sl, minlength=len(edges) - 1)
        mean = np.bincount(sl, weights=r, minlength=len(edges) - 1) / np.maximum(cnt, 1)
        lo = np.full(len(edges) - 1, np.nan)
        hi = np.full(len(edges) - 1, np.nan)
        for q in range(len(edges) - 1):
            if cnt[q]:
                lo[q], hi[q] = r[sl == q].min(), r[sl == q].max()
        out["configs"].append({"rc_min": rmin, "rc_max": rmax, "step": k,
                               "density": [round(float(c) / (Lx * Ly), 4) for c in cnt],
                               "rc_mean": [round(float(m), 4) if c else None for m, c in zip(mean, cnt)],
                               "rc_min_in_slice": [None if np.isnan(v) else round(float(v), 4) for v in lo],
                               "rc_max_in_slice": [None if np.isnan(v) else round(float(v), 4) for v in hi]})
        log(f"profile study: {rmin}/{rmax} done at step {k}")
    print(json.dumps(out), flush=True)


def speedup_study(equil: int = 5000, nsteps: int = 200):
    """DCM against a static cutoff r_c = r_c^max (Figure 38 analogue) on the thesis's slab
    geometry at its speedup-measurement size: 192,000 particles in a 76 x 76 x 44 block centred
    in 76 x 76 x 88, equilibrated `equil` Nose-Hoover steps (T* = 0.7, static r_c = 5.0). From
    that one state, each configuration runs `nsteps` timed NVE steps (after 10 untimed ones);
    reports ms per step, the force kernel's ms per launch, pairs per particle and the speedup of
    DCM over the static cutoff (which runs without interface detection)."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("thesis192k")
    t0 = time.perf_counter()
    s = dcm.System(dcm.params(st.box, rc_min=5.0, rc_max=5.0, thermostat=dcm.DCM_NOSE_HOOVER,
                              temperature=0.7, tdamp=0.5), st.x, st.v)
    for k in range(0, equil, 1000):
        s.step(min(1000, equil - k), thermo=False)
        torch.cuda.synchronize()
    s.check()
    x, v, _, _ = s.state()
    torch.cuda.synchronize()
    s.close()
    log(f"speedup study: equilibrated {equil} steps in {time.perf_counter() - t0:.1f} s")

    def run(rmin, rmax):
        # the static cutoff method has no interface detection
        de = 0 if rmin == rmax else 2
        sysm = dcm.System(dcm.params(st.box, rc_min=rmin, rc_max=rmax, detect_every=de), x, v)
        sysm.step(10, thermo=False)
        torch.cuda.synchronize()
        dcm.dcm_set_profiling(sysm.h, 2)            # events around the force launches only
        t1 = time.perf_counter()
        th = dcm.thermo_records(sysm.step(nsteps))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / nsteps
        fms, fcount = dcm.dcm_stage_times(sysm.h)["forces"]
        sysm.check()
        sysm.close()
        return ms, float(np.mean([r["pairs"] for r in th])) / st.n, fms / max(fcount, 1)

    rows = []
    static = {}
    for rmin, rmax in ((3.0, 6.0), (3.0, 7.0), (3.0, 8.0), (4.0, 8.0), (4.5, 9.5), (3.0, 10.0)):
        if rmax not in static:
            static[rmax] = run(rmax, rmax)
        ms, pp, fms = run(rmin, rmax)
        sms, spp, sfms = static[rmax]
        rows.append({"config": "DCM %.1f/%.1f" % (rmin, rmax), "ms_per_step": ms, "pairs_per_particle": pp,
                     "force_ms": fms, "static_ms_per_step": sms, "static_pairs_per_particle": spp,
                     "static_force_ms": sfms, "speedup": sms / ms, "force_speedup": sfms / fms,
                     "pair_ratio": spp / pp})
        log(f"speedup study: DCM {rmin}/{rmax}: {ms:.3f} ms (forces {fms:.3f}) vs static {sms:.3f} ms "
            f"(forces {sfms:.3f}): {sms / ms:.2f}x step, {sfms / fms:.2f}x forces, pairs {pp:.0f} vs {spp:.0f}")
    out = {"study": "speedup", "workload": "192,000 LJ particles, 76 x 76 x 44 block in 76 x 76 x 88, "
           f"NVT-equilibrated {equil} steps, then {nsteps} timed NVE steps per configuration, FP64, "
           "detect every 2nd step", "rows": rows}
    print(json.dumps(out), flush=True)


def tail_cost_study(equil: int = 100000, nsteps: int = 200):
    """Step time at matched force accuracy, with and without the runtime tail correction, on the
    thesis's geometry at 192,000 particles (the speedup study's state: NVT-equilibrated `equil`
    steps at static r_c = 5.0). The configurations pair up by their Eq. 20 error on the thesis's
    16,000-particle slab (`--accuracy-study`, 1-sigma boxes): about 0.0013-0.0015 (static 3.0
    with the correction, DCM 3.0/4.0 with it, DCM 3.0/5.0 without), about 0.0004-0.0005 (static
    4.0 and DCM 3.5/5.0 with it, DCM 3.5/5.0 without is 0.0007), and about 0.0001-0.0003 (static
    5.0, DCM 4.0/5.0 and DCM 4.5/8.0 with it; DCM 4.0/7.0 and 4.5/8.0 without). Static cutoffs
    with the correction keep the interface detection (the correction needs its fields)."""
    import numpy as np
    import torch
    from paper_1502_03234_amd import dcm, synth

    st = synth.named("thesis192k")
    s = dcm.System(dcm.params(st.box, rc_min=5.0, rc_max=5.0, thermostat=dcm.DCM_NOSE_HOOVER,
                              temperature=0.7, tdamp=0.5), st.x, st.v)
    for k in range(0, equil, 10000):
        s.step(min(10000, equil - k), thermo=False)
        torch.cuda.synchronize()
        log(f"tail cost study: equilibrated {min(k + 10000, equil)}/{equil} steps")
    s.check()
    x, v, _, _ = s.state()
    torch.cuda.synchronize()
    s.close()
    rows = []
    for rmin, rmax, tail in ((3.0, 3.0, 1), (3.0, 4.0, 1), (3.0, 5.0, 0), (4.0, 4.0, 1), (3.5, 5.0, 1),
                             (3.5, 5.0, 0), (5.0, 5.0, 1), (4.0, 5.0, 1), (4.0, 7.0, 0), (4.5, 8.0, 1),
                             (4.5, 8.0, 0)):
        de = 0 if (rmin == rmax and not tail) else 2
        sysm = dcm.System(dcm.params(st.box, rc_min=rmin, rc_max=rmax, detect_every=de, tail=tail), x, v)
        sysm.step(10, thermo=False)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        th = dcm.thermo_records(sysm.step(nsteps))
        torch.cuda.synchronize()
        ms = (time.perf_counter() - t1) * 1e3 / nsteps
        sysm.check()
        sysm.close()
        name = ("static %.1f" % rmax if rmin == rmax else "DCM %.1f/%.1f" % (rmin, rmax)) + (" + tail" if tail else "")
        pp = float(np.mean([r["pairs"] for r in th])) / st.n
        rows.append({"config": name, "ms_per_step": ms, "pairs_per_particle": pp})
        log(f"tail cost study: {name}: {ms:.3f} ms/step, {pp:.0f} pairs per particle")
    out = {"study": "tail_cost", "workload": "192,000 LJ particles, 76 x 76 x 44 block in 76 x 76 x 88, "
           f"NVT-equilibrated {equil} steps, then {nsteps} timed NVE steps per configuration, FP64",
           "rows": rows}
    print(json.dumps(out), flush=True)


def _detect_kw(args) -> dict:
    kw = dict(bin=args.study_bin, smooth_passes=args.study_smooth,
              min_component=args.study_min_component)
    if args.study_tail:
        kw["tail"] = 1
    if args.study_vapor_cutoffs:
        kw["vapor_cutoff"] = 1
    if args.study_ms_nu > 0:
        kw["ms_nu"] = args.study_ms_nu
        kw["ms_iters"] = args.study_ms_iters
    return kw


def run_study(args):
    """The studies (one per flag); each prints its own JSON line."""
    import torch

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    if args.calibrate_copy:
        src = torch.ones(args.calibrate_copy // 8, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        torch.cuda.synchronize()
        dst.copy_(src)
        torch.cuda.synchronize()
        log(f"copied {src.numel() * 8} bytes")
        return
    if args.speedup_study:
        speedup_study(args.speedup_study)
        return
    if args.profile_study:
        profile_study(args.profile_study)
        return
    if args.oracle_study:
        oracle_study()
        return
    if args.tail_cost_study:
        tail_cost_study(args.tail_cost_study)
        return
    if args.accuracy_study >= 0:
        accuracy_study(args.accuracy_study, detect_kw=_detect_kw(args))
        return
    if args.nvt_study:
        vals = [int(v) for v in args.nvt_study.split(",")]
        nvt_study(vals[0], vals[1], set(vals[2:]) or None, save_dir=args.save_dir or None,
                  detect_kw=_detect_kw(args))
        return
    if args.precision_study:
        precision_study(args.precision_study)
        return
    if args.serve:
        serving_study(args.serve, droplets=args.serve_droplets)
        return
    if args.droplet_study:
        droplet_study(args.droplet_study)
        return



def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--repeats", type=int, default=5,
                    help="timed runs of STEPS steps each; value and ms_per_step are the median run's")
    ap.add_argument("--precision", choices=["fp64", "fp32c"], default="fp64")
    ap.add_argument("--cpu-sample", type=int, default=60000)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--tail", action="store_true",
                    help="with the runtime tail correction (Eq. 21-22): its cost on the same workload")
    ap.add_argument("--skin", type=float, default=0.0,
                    help="> 0: forces from Verlet neighbour lists with this skin (Alg. 3.3)")
    ap.add_argument("--detect-every", type=int, default=2, help="re-detect the interface every k steps")
    ap.add_argument("--ms-nu", type=float, default=0.0,
                    help="segment by Eq. 13 (Mumford-Shah) with this nu instead of the threshold")
    ap.add_argument("--ms-iters", type=int, default=100, help="primal-dual iterations of --ms-nu")
    ap.add_argument("--vapor-cutoffs", action="store_true",
                    help="vapor particles with dynamic cutoffs too (Section 3.1's extension of Eq. 7)")
    ap.add_argument("--no-compare-static", action="store_true",
                    help="skip timing the same system with a static cutoff r_c = r_c^max")
    ap.add_argument("--equilibrate", type=int, default=1000,
                    help="untimed steps from the lattice start before the timed runs (steady state)")
    ap.add_argument("--serve-seeds", type=int, default=1,
                    help="serving leg of the headline line: this many Poisson traces (0: none)")
    ap.add_argument("--cpu-worker", type=str, default="", help=argparse.SUPPRESS)
    ap.add_argument("--cpu-seed", type=int, default=12345, help=argparse.SUPPRESS)
    ap.add_argument("--forces-only", type=int, default=0, metavar="K",
                    help="only create the system and run K force evaluations (counter passes)")
    ap.add_argument("--precision-study", type=int, default=0, metavar="STEPS",
                    help="256k slab: NVE drift of both forms, FP32 form force error vs the FP64 form")
    ap.add_argument("--droplet-study", type=int, default=0, metavar="STEPS",
                    help="droplet (non-planar interface) study of both forms over STEPS steps")
    ap.add_argument("--serve", type=int, default=0, metavar="SEEDS",
                    help="serving study: 64 systems, Poisson arrivals, server vs sequential")
    ap.add_argument("--serve-droplets", action="store_true",
                    help="--serve: every 4th system is a droplet instead of a slab")
    ap.add_argument("--nvt-study", type=str, default="", metavar="EQUIL,SAMPLE[,CFG...]",
                    help="Table 1 / Figure 37 observables of the thesis's 16,000-particle slab under "
                         "NVT; optional CFG indices pick Table 1 rows (0-6)")
    ap.add_argument("--accuracy-study", type=int, default=-1, metavar="EQUIL",
                    help="force accuracy (Eq. 20) of a grid of cutoff configurations against the "
                         "exact image sum, on the thesis slab after EQUIL NVT steps")
    ap.add_argument("--speedup-study", type=int, default=0, metavar="EQUIL",
                    help="DCM vs static r_c^max on the thesis's 192,000-particle slab after EQUIL steps")
    ap.add_argument("--tail-cost-study", type=int, default=0, metavar="EQUIL",
                    help="step time at matched accuracy with and without the tail correction (192k slab)")
    ap.add_argument("--oracle-study", action="store_true",
                    help="whole-run timing of the CPU oracle against the HIP path on the 16k and 256k slabs")
    ap.add_argument("--profile-study", type=int, default=0, metavar="STEPS",
                    help="cutoff profile over the density profile of the 16k slab after STEPS steps")
    ap.add_argument("--study-bin", type=float, default=1.0,
                    help="--nvt-study / --accuracy-study: density box edge (the thesis uses ~2.6)")
    ap.add_argument("--study-smooth", type=int, default=1, help="studies: smoothing passes")
    ap.add_argument("--study-min-component", type=int, default=27,
                    help="studies: components below this many boxes are removed")
    ap.add_argument("--study-ms-nu", type=float, default=0.0,
                    help="--accuracy-study / --nvt-study: Mumford-Shah segmentation (Eq. 13) with this nu")
    ap.add_argument("--study-ms-iters", type=int, default=100, help="iterations of --study-ms-nu")
    ap.add_argument("--study-vapor-cutoffs", action="store_true",
                    help="--accuracy-study / --nvt-study: vapor particles with dynamic cutoffs too")
    ap.add_argument("--study-tail", action="store_true",
                    help="--accuracy-study / --nvt-study: with the runtime tail correction (Eq. 21-22)")
    ap.add_argument("--save-dir", type=str, default="", help="--nvt-study: write the final states here")
    ap.add_argument("--calibrate-copy", type=int, default=0, metavar="BYTES",
                    help="only run one plain device copy of BYTES (HBM counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) > 1:
        print("bench.py measures one GPU only: the DCM path here has no multi-GPU "
              "decomposition; run with --gpus 1", file=sys.stderr)
        sys.exit(2)
    if args.cpu_worker:
        cpu_worker_main(args.cpu_sample, args.cpu_seed)
        return
    from paper_1502_03234_amd import synth

    studies = (args.calibrate_copy or args.speedup_study or args.profile_study or args.oracle_study
               or args.tail_cost_study or args.accuracy_study >= 0 or args.nvt_study or args.precision_study
               or args.serve or args.droplet_study)
    if studies:
        run_study(args)
        return
    log(f"generating {WORKLOAD}")
    state = synth.named(WORKLOAD)
    host = host_cpu()
    share = min(16, host["usable"])       # one GPU's share of the machine's host cores
    profiled = under_profiler()
    workers = None
    if not args.no_cpu_baseline and not profiled and share > 1:
        log(f"cpu baseline: starting {share} oracle processes (released after the GPU timing)")
        workers = cpu_workers_start(args.cpu_sample, share)

    import torch
    from paper_1502_03234_amd import dcm

    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    prec = dcm.DCM_FP64 if args.precision == "fp64" else dcm.DCM_FP32C
    p = dcm.params(state.box, precision=prec, tail=1 if args.tail else 0,
                   vapor_cutoff=1 if args.vapor_cutoffs else 0, ms_nu=args.ms_nu, ms_iters=args.ms_iters,
                   neighbor_list=1 if args.skin > 0 else 0, skin=args.skin if args.skin > 0 else 0.3,
                   detect_every=args.detect_every)
    stream = torch.cuda.current_stream()
    if args.forces_only:
        sysm = dcm.System(p, state.x, state.v)
        for _ in range(args.forces_only):
            dcm.dcm_compute_forces(sysm.h, stream)
        torch.cuda.synchronize()
        log(f"{args.forces_only} force evaluations done")
        return
    th = torch.empty(max(args.steps, args.warmup, args.equilibrate, 1) * dcm.THERMO_DOUBLES,
                     dtype=torch.float64, device=dev)
    # The lattice start roughens and its pair count grows for about a thousand steps; an untimed
    # equilibration brings the slab to that state first. Every timed run then starts from the
    # equilibrated state (positions, velocities, cutoffs, step count), takes the same W warmup
    # steps and is timed over exactly K steps; value and ms/step are the median run's. The timed
    # steps record HIP events around the force launches only (the roofline's kernel time); the
    # per-stage breakdown comes from a separate profiled run afterwards.
    eq = dcm.System(p, state.x, state.v)
    if args.equilibrate:
        log(f"equilibrating {args.equilibrate} untimed steps")
        dcm.dcm_step(eq.h, args.equilibrate, stream, th)
        torch.cuda.synchronize()
        eq.check()
    ex, ev, erc, ek = eq.state()
    torch.cuda.synchronize()
    eq.close()
    from types import SimpleNamespace
    # the state the timed runs start from, for the oracle's CPU baseline
    cpu_state = SimpleNamespace(x=ex.cpu().numpy(), v=ev.cpu().numpy(), box=state.box, n=state.n)
    runs = []
    f_ms = 0.0
    f_cnt = 0
    sysm = None
    for r in range(max(1, args.repeats)):
        if sysm is not None:
            sysm.close()
        sysm = dcm.System(p, ex, ev, rc=erc, step=ek)
        if r == 0:
            log(f"n={state.n} grid={sysm.dims} equilibrated={ek} warmup={args.warmup} repeats={args.repeats}")
        if args.warmup:
            dcm.dcm_step(sysm.h, args.warmup, stream, th)
        torch.cuda.synchronize()
        sysm.check()
        dcm.dcm_set_profiling(sysm.h, 2)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        dcm.dcm_step(sysm.h, args.steps, stream, th)
        torch.cuda.synchronize()
        runs.append(time.perf_counter() - t0)
        fst = dcm.dcm_stage_times(sysm.h)["forces"]
        f_ms += fst[0]
        f_cnt += fst[1]
    elapsed = sorted(runs)[len(runs) // 2]
    sysm.check()
    nb = max(10, args.steps // 10)
    dcm.dcm_set_profiling(sysm.h, 1)
    before = dcm.dcm_stage_times(sysm.h)
    thb = torch.empty(nb * dcm.THERMO_DOUBLES, dtype=torch.float64, device=dev)
    dcm.dcm_step(sysm.h, nb, stream, thb)
    after = dcm.dcm_stage_times(sysm.h)
    dcm.dcm_set_profiling(sysm.h, 0)
    list_builds = dcm.dcm_list_builds(sysm.h)
    rec = dcm.thermo_records(th[: args.steps * dcm.THERMO_DOUBLES])
    pairs = sum(r["pairs"] for r in rec) / len(rec)
    ms_step = elapsed / args.steps * 1e3
    value = state.n * args.steps / elapsed
    f_avg_s = f_ms / f_cnt * 1e-3
    achieved = FLOPS_PER_PAIR * pairs / f_avg_s / 1e12
    breakdown = {k: round((v[0] - before[k][0]) / nb, 5) for k, v in after.items()}
    log(f"{ms_step:.4f} ms/step, force kernel {f_avg_s * 1e3:.4f} ms, pairs/step {pairs:.4e}, "
        f"breakdown ms/step {breakdown}")
    G_boxes = int(sysm.dims[0]) * int(sysm.dims[1]) * int(sysm.dims[2])
    e0 = rec[0]["ke"] + rec[0]["pe"]
    e1 = rec[-1]["ke"] + rec[-1]["pe"]
    sysm.close()

    static = None
    if not args.no_compare_static:
        # the static cutoff method (r_c = r_c^max for every particle, no interface detection)
        # from the same equilibrated state, over the same number of steps
        ps = dcm.params(state.box, rc_min=p.rc_max, rc_max=p.rc_max, precision=prec, detect_every=0)
        ss = dcm.System(ps, ex, ev, step=ek)
        dcm.dcm_step(ss.h, max(3, args.warmup), stream, th)
        torch.cuda.synchronize()
        dcm.dcm_set_profiling(ss.h, 2)
        t0 = time.perf_counter()
        dcm.dcm_step(ss.h, args.steps, stream, th)
        torch.cuda.synchronize()
        st_ms = (time.perf_counter() - t0) / args.steps * 1e3
        sf_ms, sf_cnt = dcm.dcm_stage_times(ss.h)["forces"]
        srec = dcm.thermo_records(th[: args.steps * dcm.THERMO_DOUBLES])
        spairs = sum(r["pairs"] for r in srec) / len(srec)
        ss.check()
        ss.close()
        static = dict(r_c=p.rc_max, ms_per_step=round(st_ms, 4), dcm_speedup=round(st_ms / ms_step, 3),
                      force_ms=round(sf_ms / max(sf_cnt, 1), 4),
                      force_speedup=round(sf_ms / max(sf_cnt, 1) / (f_avg_s * 1e3), 3),
                      pairs_per_particle=round(spairs / state.n, 2),
                      pair_ratio=round(spairs / pairs, 3))
        log(f"static r_c = {p.rc_max}: {st_ms:.3f} ms/step, DCM speedup {static['dcm_speedup']}x "
            f"(forces {static['force_speedup']}x, pairs {static['pair_ratio']}x)")

    serving = None
    if args.serve_seeds > 0:
        serving = serving_study(args.serve_seeds, emit=False)

    cpu = cpu_all = None
    if not args.no_cpu_baseline:
        log(f"cpu baseline: oracle on a sample of {args.cpu_sample} particles")
        cpu = cpu_baseline(cpu_state, args.cpu_sample, total_pairs=pairs)
        if workers is not None:
            log(f"cpu baseline: releasing {share} oracle processes at once")
            path = save_state(state, cpu_state.x, cpu_state.v)
            try:
                cpu_all = cpu_workers_collect(workers, path)
            finally:
                os.unlink(path)
        elif profiled:
            cpu_all = {"skipped": "a profiler tool is loaded into this process; child processes "
                                  "would inherit it"}

    out = {
        "metric": "atom-steps/s/GPU at 2M-atom LJ slab; serving p50/p99 latency per system",
        "value": value,
        "unit": "atom-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == dcm.DCM_FP64 else "f32-compensated",
        "data": "synthetic",
        "config": {"workload": "LJ liquid/vapor slab, 2,048,000 particles, box 320x320x60, "
                               "r_c 2.5..6 (exponential), "
                               + ("detect every 2nd step" if args.detect_every == 2 else f"detect every {args.detect_every} steps")
                               + ", dt 0.005, NVE"
                               + (", runtime tail correction" if args.tail else "")
                               + (", vapor cutoffs" if args.vapor_cutoffs else "")
                               + (f", Mumford-Shah nu {args.ms_nu} x {args.ms_iters}" if args.ms_nu > 0 else "")
                               + (f", neighbour lists skin {args.skin}" if args.skin > 0 else ""),
                   "n_particles": state.n, "grid": list(sysm.dims), "detect_every": args.detect_every,
                   "thermo_every_step": True, "equilibrated_steps": int(ek),
                   "pairs_per_particle": round(pairs / state.n, 2)},
        "roofline": {"bound": "alu",
                     "kernel": ("KForces (FP64 pair forces, energy, virial; " if prec == dcm.DCM_FP64 else
                                "KForces (FP32 pair arithmetic, compensated FP32 sums, FP64 pair test; ")
                               + ("Verlet lists)" if args.skin > 0 else "rows staged in LDS)"),
                     "achieved": achieved, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                     "frac": achieved / FP64_VALU_PEAK_TFLOPS,
                     # the HBM counters were taken on the FP64 traversal kernel only
                     "traffic": force_traffic() if prec == dcm.DCM_FP64 and args.skin == 0 else None,
                     "avg_launch_ms": f_avg_s * 1e3, "pairs_per_launch": pairs,
                     "flops_per_pair": FLOPS_PER_PAIR},
        "cpu_baseline": cpu and dict({k: cpu[k] for k in ("value", "unit", "cores", "kind", "sample")},
                                     host=host, extrapolation_by_pairs=cpu.get("by_pairs")),
        "cpu_baseline_all_cores": cpu_all,
        "breakdown_ms_per_step": breakdown,
        "stage_bandwidth": stage_bandwidth(breakdown, state.n, G_boxes, args.detect_every),
        "energy_drift_per_atom": (e1 - e0) / state.n,
        "static_cutoff_6": static,
        "serving": serving and {
            "workload": f"{serving['systems']} slab systems of 4,000-200,000 particles, "
                        f"{serving['steps_each']} steps each, Poisson arrivals at {serving['load']} of the "
                        f"sequential capacity, {serving['seeds']} trace",
            "server": serving["server"], "sequential": serving["sequential"],
            "saturated_atom_steps_per_s": {"server": serving["saturated"]["server_atom_steps_per_s"],
                                           "sequential": serving["saturated"]["sequential_atom_steps_per_s"]}},
        "timing": {"repeats": len(runs), "of_steps": args.steps, "statistic": "median",
                   "ms_per_step_runs": [round(r / args.steps * 1e3, 4) for r in runs]},
    }
    if args.skin > 0:
        out["neighbour_lists"] = {"skin": args.skin, "builds": list_builds,
                                  "steps_run": args.warmup + args.steps + nb}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
