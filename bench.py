"""Benchmark of the EAM timestep loop on one MI355X.

Headline: the 128,000-atom BCC box (40^3 cells, a = 3.304 A), float64, 300 K,
skin 0.3 A, dt = 1 fs; W untimed warm-up steps, then exactly K timed steps,
every one of them inside a captured hipGraph (100-step chunks, the left-over
steps as one shorter graph).  Prints one JSON line: timesteps/s, atom-steps/s,
the roofline of the dominant kernel (force pass fused with the integration),
the measured copy bandwidth, and the secondary workloads:
  c1_2000          2,000 atoms, float64, 100 steps (launch-latency regime)
  c2_10000         128,000 atoms, 10,000 steps in 100-step graph chunks:
                   per-chunk timesteps/s, mean list length and temperature,
                   energy drift
  c3_810k          802,344 atoms, float64 and mixed precision, 5,000 steps;
                   mixed forces at steps 0, 1000, ..., 5000
  slab_801792      the paper-shaped 256 x 261 x 6 slab, open in x and y
  half_list_128k   force symmetry (each pair evaluated once)
  alloy_128k       two atom types
  perf_model       t = A n_cand + B n_int + C with the candidate filter run
                   every step, and the list-reuse form
  batched_256      256 replicas in one launch per pass vs a sequential loop
  force_matching   gradient evaluations/s of the adjoint
and the CPU-oracle leg (cpu_baseline): the FP64 oracle timed on the host on
each workload's sample, and the mixed-precision force error against it.

Usage: python bench.py [--gpus 1] [--steps 10000] [--warmup 100]
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

METRIC = "timesteps/s and atom-steps/s, EAM BCC 128k & 810k atoms, FP64 vs mixed"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
CSRC = os.path.join(ROOT, "paper_2405_07898_amd", "csrc")
# the sources that define the dominant kernel (its counters go stale when any changes)
TRAFFIC_SOURCES = ("md_kernels.hip", "md_device.h", "md_internal.h")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_integrate_128k_traffic.json")
CHUNK = 100
# re-sort atoms by cell every 2 graph chunks (200 steps): the specified potential's
# lattice melts and its atoms diffuse, so the cell order of the slots decays
# (measured at 128,000 atoms: 55.6 us/step re-sorting every 2 chunks against
# 59.9 every 10)
SORT_EVERY = 2
SECTIONS = ("c1", "c2", "c3", "slab", "half", "alloy", "perf_model", "batched", "fm")


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def force_pass_bytes(n_atoms: int, n_l: float, mixed: bool) -> float:
    """Algorithmic HBM bytes of one force+integrate launch.

    Per atom: x (24) + F' (8) + list length (4) + list entries (4 n_l) + v read
    and write (48) + new x (24) + x_ref (24) = 132 + 4 n_l; the unfused pair
    (force 60 + 4 n_l, integration 144) less the force written and read back
    and x read again.  The mixed form reads the atom's 16-byte record
    (fixed-point position and F') in place of F' and writes the record of the
    new position: 156 + 4 n_l.  Neighbour gathers are cache-served and not
    counted.
    """
    per = (24 + 8 + 4 + 4 * n_l + 48 + 24 + 24) if not mixed else \
        (24 + 16 + 4 + 4 * n_l + 48 + 24 + 16 + 24)
    return n_atoms * per


def density_pass_bytes(n_atoms: int, n_l: float, mixed: bool = False) -> float:
    """Algorithmic bytes of one density launch: x (24) + list length (4) + list
    entries (4 n_l) + F' written (8) = 36 + 4 n_l per atom.  The mixed form
    reads the atom's 16-byte record in place of x and also writes F' into it
    (4): 32 + 4 n_l."""
    return n_atoms * ((16 + 4 + 8 + 4 if mixed else 24 + 4 + 8) + 4 * n_l)

def force_pass_flops(n_atoms: int, n_l: float, n_int: float) -> float:
    """Algorithmic flops (paper Table "flopmodel"): 9 per list entry (distance and
    test), 31 per interaction (r^-1, r, segment, rho' and phi', force), 8 per atom
    (F' sum reuse and the Verlet update)."""
    return n_atoms * (9 * n_l + 31 * n_int + 8)


def source_hash() -> str:
    h = hashlib.sha256()
    for name in TRAFFIC_SOURCES:
        with open(os.path.join(CSRC, name), "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def load_traffic(n_atoms: int, n_l: float, lpa: int):
    """HBM bytes per launch of the dominant kernel from the committed rocprofv3
    counter runs, if they were taken on the current kernel sources, at the same
    atom count and lanes per atom and at a mean list length within 2 % of this
    state's; else None with the reason."""
    if not os.path.exists(TRAFFIC_FILE):
        return None, "no counter file"
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != source_hash():
        return None, "kernel sources changed since the counters were taken"
    for e in t.get("entries", []):
        if (e.get("n_atoms") == n_atoms and e.get("lanes_per_atom") == lpa
                and abs(e.get("mean_list_length", -1.0) - n_l) <= 0.02 * n_l):
            return e.get("bytes_per_launch"), t.get("summary")
    return None, "no counter run at this atom count and list length"


def launch_plan(parity: int, steps: int, chunk: int = CHUNK):
    """The graph launches md_step makes for `steps` steps starting on position
    buffer `parity` (whole chunks from buffer 0, the rest as shorter graphs of
    at most chunk - 1 steps)."""
    chunks, tails, done = 0, [], 0
    while done < steps:
        if parity == 0 and steps - done >= chunk:
            chunks += 1
            done += chunk
        else:
            n = min(steps - done, chunk - 1)
            tails.append(n)
            parity ^= n & 1
            done += n
    return {"chunk_graphs": chunks, "chunk_steps": chunk, "shorter_graphs": tails}


def make_params(md, *, precision, chunk=CHUNK, lpa=0, **kw):
    from workloads import configs, potential

    base = dict(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=configs.SKIN,
                ftm2v=configs.FTM2V, precision=precision, chunk_steps=chunk,
                lanes_per_atom=lpa, nbr_capacity=128, cell_capacity=64, sort_every=SORT_EVERY)
    base.update(kw)
    return md.make_params(**base)


def make_system(md, box, tabs, *, precision, chunk=CHUNK, lpa=0, **kw):
    p = make_params(md, precision=precision, chunk=chunk, lpa=lpa, **kw)
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    return s


def time_steps(torch, s, steps: int):
    """Seconds for `steps` MD steps (events on the library stream), bracketed
    by device synchronisations; and the host wall time."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s.prepare(steps)  # graphs captured outside the timed region
    torch.cuda.synchronize()
    s.stream.synchronize()
    t0 = time.perf_counter()
    e0.record(s.stream)
    s.step(steps)
    e1.record(s.stream)
    s.stream.synchronize()
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ev = e0.elapsed_time(e1) * 1e-3
    return max(ev, 1e-12), wall


def time_kernel(torch, s, md, which: int, reps: int) -> float:
    """Average duration (us) of one pass kernel: `reps` back-to-back launches on
    the library's stream between one pair of events, divided by `reps`."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    s.launch_pass(which, 2)  # warm
    s.stream.synchronize()
    e0.record(s.stream)
    s.launch_pass(which, reps)
    e1.record(s.stream)
    s.stream.synchronize()
    return e0.elapsed_time(e1) * 1e3 / reps


def temperature(ke: float, n: int) -> float:
    from workloads import configs

    return 2.0 * ke / (max(3 * n - 3, 1) * configs.KBOLTZ)


def copy_probe(torch, mib: int, reps: int = 5) -> dict:
    """A plain elementwise copy (y = -x, float64) of known size: it reads and
    writes mib MiB once per launch.  Its rate is the achievable-HBM reference,
    and hardware byte counters read on it give the factor between counter
    units and bytes moved."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.neg(src, out=dst)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    del src, dst
    return {"bytes_read": n * 8, "bytes_written": n * 8, "launches": reps,
            "avg_us": round(us, 2), "gbs": round(2 * n * 8 / (us * 1e-6) / 1e9, 1)}


# ------------------------------------------------------------------- headline

def bench_headline(torch, md, configs, tabs, args, copy_gbs):
    box = configs.config_128k() if args.workload == "128k" else configs.config_810k()
    log(f"workload {args.workload}: n={box.n}; building")
    s = make_system(md, box, tabs, precision=md.MD_FP64, lpa=args.lpa)
    if args.lpa == 0:
        lpa, us = s.autotune(50)
        log(f"autotune: {lpa} lanes per atom ({us:.1f} us per density+force)")
    else:
        lpa = args.lpa
    pe0, ke0 = s.energy()
    log(f"warmup {args.warmup} steps")
    s.step(args.warmup)
    st0 = s.stats()
    plan = launch_plan(args.warmup & 1, args.steps)
    log(f"timing {args.steps} steps ({plan})")
    sec, wall = time_steps(torch, s, args.steps)
    st1 = s.stats()
    pe1, ke1 = s.energy()
    ts = args.steps / sec
    n_l = st1["list_entries"] / box.n
    log(f"{ts:.1f} timesteps/s ({sec * 1e3 / args.steps:.4f} ms/step, wall {wall:.3f} s), "
        f"rebuilds {st1['rebuilds'] - st0['rebuilds']}, mean list {n_l:.2f}")
    # the dominant kernel at the state the timed steps ended in, on the library stream
    dens_us = time_kernel(torch, s, md, md.PASS_DENSITY, args.kernel_reps)
    force_us = time_kernel(torch, s, md, md.PASS_FORCE_RAW, args.kernel_reps)
    s.close()
    byts = force_pass_bytes(box.n, n_l, False)
    flops = force_pass_flops(box.n, n_l, n_l)
    gbs = byts / (force_us * 1e-6) / 1e9
    tfl = flops / (force_us * 1e-6) / 1e12
    dbytes = density_pass_bytes(box.n, n_l)
    # the roofline that binds: intensity below the float64 ridge -> HBM
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    bound = "hbm" if flops / byts < ridge else "alu"
    traffic, traffic_note = load_traffic(box.n, n_l, lpa)
    roof = {"bound": bound, "kernel": "k_force_integrate<fp64>",
            "achieved": round(gbs, 1) if bound == "hbm" else round(tfl, 3),
            "peak": HBM_PEAK_GBS if bound == "hbm" else FP64_PEAK_TFLOPS,
            "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
            "frac": round((gbs / HBM_PEAK_GBS) if bound == "hbm" else (tfl / FP64_PEAK_TFLOPS), 4),
            "traffic": traffic, "traffic_note": traffic_note,
            "algorithmic_bytes_per_launch": byts, "bytes_per_atom": "132 + 4 n_l",
            "algorithmic_flops_per_launch": flops, "avg_kernel_us": round(force_us, 3),
            "frac_of_measured_copy": round(gbs / copy_gbs, 4) if copy_gbs else None,
            "alu_frac": round(tfl / FP64_PEAK_TFLOPS, 4), "mean_list_length": round(n_l, 3),
            "density_kernel_us": round(dens_us, 3),
            "density_hbm_frac": round(dbytes / (dens_us * 1e-6) / 1e9 / HBM_PEAK_GBS, 4)}
    log(f"force pass {force_us:.2f} us -> {gbs:.0f} GB/s ({roof['frac'] * 100:.1f}% HBM), "
        f"{tfl:.2f} TFLOP/s; density {dens_us:.2f} us")
    start = "from the 300 K lattice" if args.warmup == 0 else \
        f"after {args.warmup} warm-up steps from the 300 K lattice"
    out = {
        "metric": METRIC, "value": round(ts, 2), "unit": "timesteps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3 / args.steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload] + f"; {args.steps} timed steps {start}",
                   "n_atoms": box.n, "launch": "hipGraph", **plan, "lanes_per_atom": lpa},
        "atom_steps_per_s": round(ts * box.n, 1),
        "energy_drift_per_atom_eV": float(abs((pe1[0] + ke1[0]) - (pe0[0] + ke0[0])) / box.n),
        "rebuilds_in_timed_region": int(st1["rebuilds"] - st0["rebuilds"]),
        "mean_list_length": round(n_l, 3),
        "wall_s_timed": round(wall, 4),
        "roofline": roof,
    }
    return out, box


# ------------------------------------------------------------------ secondaries

def bench_c1(torch, md, configs, tabs, persistent=True, lpa=0):
    """2,000-atom box (launch-latency regime): 100 steps as one captured graph
    from the prepared state (the workload's own length), a longer 2,000-step
    window, and one persistent cooperative launch per chunk for comparison
    (skipped with persistent=False: rocprofv3 ends with a segmentation fault
    after cooperative launches, before it writes its results)."""
    box = configs.config_small()
    if lpa <= 0:
        s = make_system(md, box, tabs, precision=md.MD_FP64)
        lpa, _ = s.autotune(50)
        s.close()
    s = make_system(md, box, tabs, precision=md.MD_FP64, lpa=lpa)
    pe0, ke0 = s.energy()
    sec100, _ = time_steps(torch, s, 100)  # one 100-step graph from the prepared state
    pe1, ke1 = s.energy()
    sec, _ = time_steps(torch, s, 2000)
    st = s.stats()
    s.close()
    sec_p = None
    if persistent:
        sp = make_system(md, box, tabs, precision=md.MD_FP64, lpa=8,
                         launch_mode=md.MD_LAUNCH_PERSISTENT)
        sp.step(100)
        sec_p, _ = time_steps(torch, sp, 2000)
        sp.close()
    return {"n_atoms": box.n, "lanes_per_atom": lpa,
            "steps_100": {"timesteps_per_s": round(100 / sec100, 1),
                          "atom_steps_per_s": round(100 / sec100 * box.n, 1),
                          "energy_drift_per_atom_eV": float(abs((pe1[0] + ke1[0])
                                                                - (pe0[0] + ke0[0])) / box.n)},
            "steps_2000": {"timesteps_per_s": round(2000 / sec, 1),
                           "atom_steps_per_s": round(2000 / sec * box.n, 1),
                           "us_per_step": round(sec / 2000 * 1e6, 3)},
            "rebuilds": st["rebuilds"],
            "persistent_launch_timesteps_per_s": round(2000 / sec_p, 1) if sec_p else None}


def bench_c2_series(torch, md, configs, tabs, steps=10000):
    """The 128,000-atom workload as specified: 10,000 steps from the 300 K
    lattice in 100-step graph chunks, each chunk timed with events on the
    library stream; after each chunk the mean list length of the last build
    and the temperature.  Energy drift over the whole run."""
    box = configs.config_128k()
    s = make_system(md, box, tabs, precision=md.MD_FP64)
    lpa, _ = s.autotune(50)
    s.close()
    s = make_system(md, box, tabs, precision=md.MD_FP64, lpa=lpa)
    pe0, ke0 = s.energy()
    e = [torch.cuda.Event(enable_timing=True) for _ in range(2)]
    chunk_ms, n_l, temp, etot = [], [], [], []
    st_prev = s.stats()
    rebuilds = []
    s.prepare(CHUNK)
    for _ in range(steps // CHUNK):
        s.stream.synchronize()
        e[0].record(s.stream)
        s.step(CHUNK)
        e[1].record(s.stream)
        s.stream.synchronize()
        chunk_ms.append(e[0].elapsed_time(e[1]))
        st = s.stats()
        n_l.append(st["list_entries"] / box.n)
        rebuilds.append(int(st["rebuilds"] - st_prev["rebuilds"]))
        st_prev = st
        pe, ke = s.energy()
        temp.append(temperature(ke[0], box.n))
        etot.append(pe[0] + ke[0])
    s.close()
    total_s = sum(chunk_ms) * 1e-3
    e0 = pe0[0] + ke0[0]
    per_chunk = [CHUNK / (ms * 1e-3) for ms in chunk_ms]
    return {"n_atoms": box.n, "steps": steps, "lanes_per_atom": lpa,
            "timesteps_per_s": round(steps / total_s, 1),
            "atom_steps_per_s": round(steps / total_s * box.n, 1),
            "median_chunk_timesteps_per_s": round(float(np.median(per_chunk)), 1),
            "energy_drift_per_atom_eV": float(abs(etot[-1] - e0) / box.n),
            "max_energy_deviation_per_atom_eV": float(np.max(np.abs(np.array(etot) - e0)) / box.n),
            "rebuilds": int(sum(rebuilds)),
            "series": {"chunk_timesteps_per_s": [round(v, 1) for v in per_chunk],
                       "mean_list_length": [round(v, 3) for v in n_l],
                       "temperature_K": [round(v, 1) for v in temp],
                       "rebuilds": rebuilds}}


def bench_c3(torch, md, configs, tabs, args):
    """802,344 atoms (74^3 sites, 1 % vacancies, 2,500 K): the float64 and the
    mixed form, 5,000 steps each.  The mixed run pauses every 1,000 steps
    (untimed) to export its positions and its forces there, and the float64
    path's forces on the same positions; the oracle's forces on them come in
    the CPU leg."""
    big = configs.config_810k()
    steps = args.secondary_steps
    snap_every = max(steps // 5, 1)
    out = {"n_atoms": big.n, "steps": steps,
           "workload": "74^3 BCC sites - 1% vacancies, 2500 K"}
    snaps = []
    s64_eval = None
    for name, prec in (("fp64", md.MD_FP64), ("mixed", md.MD_MIXED)):
        log(f"c3 {name}: n={big.n}")
        lpa = args.lpa
        if args.lpa == 0:
            # tuned on a copy of the box after 200 steps: the timed run spends
            # almost all its steps in the hot, disordered state, not the lattice
            sw = make_system(md, big, tabs, precision=prec, lpa=2)
            sw.step(200)
            lpa, us = sw.autotune(20)
            sw.close()
            log(f"  autotune (after 200 steps): {lpa} lanes per atom ({us:.1f} us per density+force)")
        sb = make_system(md, big, tabs, precision=prec, lpa=lpa)
        st0 = sb.stats()
        total = 0.0
        done = 0
        while done < steps:
            if name == "mixed" and done % snap_every == 0:
                snaps.append(_c3_snapshot(torch, md, sb, big, tabs, done, s64_eval))
            n = min(snap_every, steps - done)
            t, _ = time_steps(torch, sb, n)
            total += t
            done += n
        if name == "mixed":
            snaps.append(_c3_snapshot(torch, md, sb, big, tabs, done, s64_eval))
        stb = sb.stats()
        nlb = stb["list_entries"] / big.n
        fu = time_kernel(torch, sb, md, md.PASS_FORCE_RAW, 50)
        du = time_kernel(torch, sb, md, md.PASS_DENSITY, 50)
        b2 = force_pass_bytes(big.n, nlb, prec == md.MD_MIXED)
        out[name] = {"timesteps_per_s": round(steps / total, 2),
                     "atom_steps_per_s": round(steps / total * big.n, 1),
                     "lanes_per_atom": lpa,
                     "force_pass_us": round(fu, 3),
                     "force_pass_hbm_frac": round(b2 / (fu * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                     "density_pass_us": round(du, 3),
                     "density_pass_hbm_frac": round(density_pass_bytes(big.n, nlb, prec == md.MD_MIXED) / (du * 1e-6)
                                                    / 1e9 / HBM_PEAK_GBS, 4),
                     "mean_list_length": round(nlb, 3),
                     "rebuilds": int(stb["rebuilds"] - st0["rebuilds"])}
        sb.close()
        if name == "fp64":
            # a float64 context that evaluates forces on the mixed run's positions
            s64_eval = md.System(make_params(md, precision=md.MD_FP64, sort_every=0), tabs,
                                 [big.n], big.box[None, :])
        log(f"  {out[name]}")
    s64_eval.close()
    out["mixed_over_fp64"] = round(out["mixed"]["timesteps_per_s"]
                                   / out["fp64"]["timesteps_per_s"], 4)
    return out, big, snaps


def _c3_snapshot(torch, md, sm, box, tabs, step, s64):
    """Positions of the mixed run at `step`, its mixed forces there, and the
    float64 path's forces on the same positions."""
    x, _, _ = sm.get_state(want_f=False)
    fm, _, _ = sm.compute_forces()
    s64.set_state(x, torch.zeros_like(x))
    s64.build_neighbors()
    f64, _, _ = s64.compute_forces()
    return {"step": step, "x": x.cpu().numpy(), "f_mixed": fm.cpu().numpy(),
            "f_fp64": f64.cpu().numpy()}


def bench_slab(torch, md, configs, tabs, steps):
    """The paper's benchmark geometry (Sec. IV-B): an 801,792-atom BCC slab of
    256 x 261 x 6 cells, open in x and y, periodic through its thickness, at
    300 K, with the specified potential."""
    box = configs.config_slab_801792()
    s = make_system(md, box, tabs, precision=md.MD_FP64)
    lpa, _ = s.autotune(20)
    s.step(100)
    st0 = s.stats()
    sec, _ = time_steps(torch, s, steps)
    st1 = s.stats()
    s.close()
    return {"workload": "BCC slab 256x261x6 cells, open x/y, periodic z, 300 K",
            "n_atoms": box.n, "steps": steps, "lanes_per_atom": lpa,
            "timesteps_per_s": round(steps / sec, 1),
            "atom_steps_per_s": round(steps / sec * box.n, 1),
            "rebuilds": int(st1["rebuilds"] - st0["rebuilds"]),
            "mean_list_length": round(st1["list_entries"] / box.n, 3)}


def bench_half(torch, md, configs, tabs, steps):
    """Force symmetry: the 128,000-atom workload with the half-list form (each
    pair evaluated once, two-phase deterministic reduction), against the
    full-list form on the same box and schedule."""
    box = configs.config_128k()
    out = {"n_atoms": box.n, "steps": steps}
    for name, mode in (("full", md.MD_LIST_FULL), ("half", md.MD_LIST_HALF)):
        s = make_system(md, box, tabs, precision=md.MD_FP64, list_mode=mode)
        lpa, _ = s.autotune(20)
        s.step(100)
        st0 = s.stats()
        sec, _ = time_steps(torch, s, steps)
        st1 = s.stats()
        dens = time_kernel(torch, s, md, md.PASS_DENSITY, 50)
        frc = time_kernel(torch, s, md, md.PASS_FORCE_RAW, 50)
        s.close()
        out[name] = {"timesteps_per_s": round(steps / sec, 1), "lanes_per_atom": lpa,
                     "density_pass_us": round(dens, 3), "force_pass_us": round(frc, 3),
                     "rebuilds": int(st1["rebuilds"] - st0["rebuilds"]),
                     "mean_list_length": round(st1["list_entries"] / box.n, 3)}
    return out


def bench_alloy(torch, md, configs, potential, steps):
    """Several atom types: the 128,000-atom random equiatomic binary alloy (per-type
    rho and F, per-pair phi, per-type masses), same schedule as the main workload."""
    box = configs.config_alloy_128k()
    p = make_params(md, precision=md.MD_FP64, n_types=2)
    s = md.System(p, potential.alloy_tables(), [box.n], box.box[None, :],
                  masses=potential.ALLOY_MASS)
    s.set_state(box.x, box.v)
    s.set_types(box.types)
    s.build_neighbors()
    lpa, _ = s.autotune(20)
    s.step(100)
    st0 = s.stats()
    sec, _ = time_steps(torch, s, steps)
    st1 = s.stats()
    dens = time_kernel(torch, s, md, md.PASS_DENSITY, 50)
    frc = time_kernel(torch, s, md, md.PASS_FORCE_RAW, 50)
    s.close()
    return {"workload": "random equiatomic binary BCC alloy, 40^3 cells, 300 K",
            "n_atoms": box.n, "n_types": 2, "steps": steps, "lanes_per_atom": lpa,
            "timesteps_per_s": round(steps / sec, 1),
            "density_pass_us": round(dens, 3), "force_pass_us": round(frc, 3),
            "rebuilds": int(st1["rebuilds"] - st0["rebuilds"]),
            "mean_list_length": round(st1["list_entries"] / box.n, 3)}


def _candidates_per_atom(box, rl):
    """Mean number of atoms in the 27 cells around each atom's cell (itself
    included): the candidates the list build tests."""
    L = box.box
    nc = np.floor(L / rl).astype(np.int64)
    c = np.minimum((box.x * (nc / L)).astype(np.int64), nc - 1)
    flat = (c[:, 2] * nc[1] + c[:, 1]) * nc[0] + c[:, 0]
    occ = np.bincount(flat, minlength=int(np.prod(nc))).reshape(nc[2], nc[1], nc[0])
    s = np.zeros_like(occ)
    for dz in (-1, 0, 1):
        for dy in (-1, 0, 1):
            for dx in (-1, 0, 1):
                s += np.roll(occ, (dz, dy, dx), axis=(0, 1, 2))
    return float((occ * s).sum() / box.n)


def _fit(rows, cols, target):
    m = np.array(rows)
    X = np.column_stack([m[:, c] for c in cols] + [np.ones(len(m))])
    coef, *_ = np.linalg.lstsq(X, m[:, target], rcond=None)
    pred = X @ coef
    r2 = 1.0 - np.sum((m[:, target] - pred) ** 2) / np.sum((m[:, target] - m[:, target].mean()) ** 2)
    return coef, float(r2)


def perf_model(torch, md, configs, tabs, steps: int = 1000, reps: int = 20):
    """Linear models of the step time at fixed N (the paper's Eq. linearmodel /
    Table "regression": t = A n_cand + B n_int + C), from dt = 0 sweeps of the
    interaction cutoff and the skin on the 128,000-atom lattice.

    - every_step: the candidate filter runs every step, as on the wafer: binning
      + list build + density + force (each kernel timed over `reps`
      back-to-back launches), fitted to candidates and interactions per atom;
    - list_reuse: md_step with the list kept (dt = 0 never triggers a rebuild),
      fitted to list entries and interactions per atom."""
    from workloads import potential

    box = configs.config_128k()
    rows = []
    for rc in (3.0, 3.5, 4.0, 5.0):
        for skin in (0.3, 0.8, 1.4, 2.2):
            p = md.make_params(mass=configs.MASS, dt=0.0, r_cut=rc, skin=skin,
                               ftm2v=configs.FTM2V, precision=md.MD_FP64, chunk_steps=CHUNK,
                               lanes_per_atom=2, nbr_capacity=160, cell_capacity=64,
                               sort_every=0)
            s = md.System(p, tabs, [box.n], box.box[None, :])
            s.set_state(box.x, box.v)
            s.build_neighbors()
            s.step(200)
            sec, _ = time_steps(torch, s, steps)
            n_l = s.stats()["list_entries"] / box.n
            t_build = time_kernel(torch, s, md, md.PASS_BUILD, reps)
            t_bin1 = time_kernel(torch, s, md, md.PASS_BIN, reps)  # reps binnings + one build
            t_bin = t_bin1 - t_build / reps
            t_dens = time_kernel(torch, s, md, md.PASS_DENSITY, reps)
            t_frc = time_kernel(torch, s, md, md.PASS_FORCE_RAW, reps)
            cnt, nbr = s.neighbors(160)
            s.close()
            # interactions (r < r_cut) of a fixed sample of atoms, from the exported list
            pick = np.random.default_rng(9).choice(box.n, 4096, replace=False)
            c = cnt.cpu().numpy()[pick]
            nb = nbr.cpu().numpy()[pick]
            n_int = 0
            for a, ca, na in zip(pick, c, nb):
                d = box.x[na[:ca]] - box.x[a]
                d -= box.box * np.round(d / box.box)
                n_int += int(np.count_nonzero((d * d).sum(1) < rc * rc))
            n_c = _candidates_per_atom(box, rc + skin)
            cells = float(np.prod(np.floor(box.box / (rc + skin))))
            rows.append((n_c, n_l, n_int / len(pick), t_bin + t_build + t_dens + t_frc,
                         sec / steps * 1e6, rc, skin, t_build, t_bin, t_dens, t_frc,
                         cells / box.n))
    ce, r2e = _fit(rows, (0, 2), 3)
    cg, r2g = _fit(rows, (0, 2, 11), 3)
    cr, r2r = _fit(rows, (1, 2), 4)
    ns = 1e3 / box.n  # us per step -> ns per atom-step
    return {"n_atoms": box.n, "lanes_per_atom": 2,
            "every_step": {"us_per_step_per_candidate": round(float(ce[0]), 5),
                           "us_per_step_per_interaction": round(float(ce[1]), 5),
                           "us_per_step_fixed": round(float(ce[2]), 3),
                           "ns_per_atom_candidate": round(float(ce[0]) * ns, 7),
                           "ns_per_atom_interaction": round(float(ce[1]) * ns, 7),
                           "ns_per_atom_fixed": round(float(ce[2]) * ns, 6), "r2": round(r2e, 5)},
            # the list build takes one wave per cell: a per-cell term besides the paper's
            "every_step_with_cells": {"us_per_step_per_candidate": round(float(cg[0]), 5),
                                      "us_per_step_per_interaction": round(float(cg[1]), 5),
                                      "us_per_step_per_cell_per_atom": round(float(cg[2]), 3),
                                      "ns_per_cell": round(float(cg[2]) * ns, 5),
                                      "us_per_step_fixed": round(float(cg[3]), 3),
                                      "r2": round(r2g, 5)},
            "list_reuse": {"us_per_step_per_list_entry": round(float(cr[0]), 5),
                           "us_per_step_per_interaction": round(float(cr[1]), 5),
                           "us_per_step_fixed": round(float(cr[2]), 3), "r2": round(r2r, 5)},
            "paper_wse_ns": {"candidate": 26.6, "interaction": 71.4, "fixed": 574},
            "points": [{"r_cut": r[5], "skin": r[6], "n_cand": round(r[0], 2),
                        "n_l": round(r[1], 3), "n_int": round(r[2], 3),
                        "us_every_step": round(r[3], 3), "us_list_reuse": round(r[4], 3),
                        "us_build": round(r[7], 3), "us_bin": round(r[8], 3),
                        "us_density": round(r[9], 3), "us_force": round(r[10], 3),
                        "cells": round(r[11] * box.n)}
                       for r in rows]}


def bench_batched(torch, md, configs, tabs, args):
    """256 replicas (5-20 cells, 0-2 % vacancies, 300-2000 K) in one launch per pass,
    against a sequential loop of single-replica contexts."""
    reps = configs.config_batch(256)
    n_tot = sum(b.n for b in reps)
    res = {"n_replicas": len(reps), "n_atoms_total": n_tot}
    sizes = np.array([b.n for b in reps])
    cls = np.where(sizes <= 2048, 0, np.where(sizes <= 8192, 1, 2))
    x0 = np.concatenate([b.x for b in reps])
    v0 = np.concatenate([b.v for b in reps])

    def fresh(p):
        s = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
        s.set_state(x0, v0)
        s.build_neighbors()
        return s

    steps = args.batched_steps
    for name, prec in (("fp64", md.MD_FP64), ("mixed", md.MD_MIXED)):
        p = make_params(md, precision=prec, sort_every=1)
        s = fresh(p)
        lpa, us = s.autotune(20)
        sched = s.replica_schedule()
        s.close()
        res[name] = {"steps": steps, "lanes_per_atom_uniform_best": lpa,
                     "lanes_per_atom_by_size_class": {
                         c: int(sched[cls == k][0]) for k, c in
                         enumerate(("<=2048 atoms", "<=8192 atoms", ">8192 atoms"))
                         if np.any(cls == k)}}
        # the autotuned schedule and the single best value for all, each from the
        # same initial state over the same steps
        for mode, set_sched in (("autotuned", lambda q: q.set_replica_schedule(sched)),
                                ("uniform", lambda q: q.set_schedule(lpa))):
            s = fresh(p)
            set_sched(s)
            s.step(100)
            sec, _ = time_steps(torch, s, steps)
            s.close()
            res[name][mode] = {"timesteps_per_s": round(steps / sec, 2),
                               "atom_steps_per_s": round(steps * n_tot / sec, 1)}
        res[name]["timesteps_per_s"] = res[name]["autotuned"]["timesteps_per_s"]
        res[name]["atom_steps_per_s"] = res[name]["autotuned"]["atom_steps_per_s"]
    # sequential per-replica loop (float64), same kernels, one context per replica
    seq_steps = args.sequential_steps
    systems = []
    for b in reps:
        s = make_system(md, b, tabs, precision=md.MD_FP64, chunk=50, sort_every=1)
        s.step(50)
        systems.append(s)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s in systems:
        s.step(seq_steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    for s in systems:
        s.close()
    res["sequential_fp64"] = {"steps_per_replica": seq_steps,
                              "atom_steps_per_s": round(seq_steps * n_tot / sec, 1)}
    res["batched_over_sequential_fp64"] = round(
        res["fp64"]["atom_steps_per_s"] / res["sequential_fp64"]["atom_steps_per_s"], 2)
    return res


def bench_fm(torch, md, configs, potential, tabs):
    """Force-matching gradient evaluations (forward + adjoint) over 64 x 2,000 atoms."""
    from paper_2405_07898_amd import fm

    boxes = configs.config_fm(64, 10)
    x = np.concatenate([b.x for b in boxes])
    # reference forces from the library's float64 pass with the 2000-knot tables
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=0.0,
                       ftm2v=configs.FTM2V)
    s = md.System(p, tabs, [b.n for b in boxes], np.stack([b.box for b in boxes]))
    s.set_state(x, np.zeros_like(x))
    s.build_neighbors()
    fref, _, _ = s.compute_forces()
    s.close()
    ftabs = potential.fm_tables()
    prob = fm.ForceMatch(x, fref, [b.n for b in boxes], np.stack([b.box for b in boxes]), ftabs)
    coefs = [torch.as_tensor(t.coef, device="cuda") for t in ftabs]
    for _ in range(3):
        prob.forward(*coefs)
        prob.backward()
    reps = 50
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.forward(*coefs)
        prob.backward()
    torch.cuda.synchronize()
    sec_sync = time.perf_counter() - t0
    # the device-resident loop an optimiser runs: no host round trip per
    # evaluation, one status check at the end
    one = torch.ones((), dtype=torch.float64, device="cuda")
    for _ in range(3):
        prob.forward_async(*coefs)
        prob.backward_async(one)
    prob.check()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        prob.forward_async(*coefs)
        prob.backward_async(one)
    prob.check()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    prob.close()
    problem = {"x": x, "fref": fref.cpu().numpy(), "boxes": np.stack([b.box for b in boxes]),
               "offsets": np.concatenate([[0], np.cumsum([b.n for b in boxes])]), "tabs": ftabs}
    return {"n_configs": 64, "n_atoms_total": int(x.shape[0]),
            "gradient_evaluations_per_s": round(reps / sec, 2),
            "ms_per_gradient_evaluation": round(sec / reps * 1e3, 4),
            "with_host_sync_each_evaluation": {
                "gradient_evaluations_per_s": round(reps / sec_sync, 2),
                "ms_per_gradient_evaluation": round(sec_sync / reps * 1e3, 4)}}, problem


# ------------------------------------------------------------- CPU oracle leg

def cpu_baseline(box, tabs, budget_s: float = 15.0):
    """The FP64 oracle on the headline workload: OpenMP over atoms on the
    host's cores, then a shorter single-thread sample."""
    import oracle
    from workloads import configs, potential

    oracle.build(force=False)
    threads = oracle.get_threads()
    kw = dict(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=configs.SKIN,
              ftm2v=configs.FTM2V)
    t0 = time.perf_counter()
    oracle.md_run(box.x, box.v, box.box, tabs, 5, **kw)
    per = (time.perf_counter() - t0) / 5.0
    steps = int(max(5, min(2000, budget_s / max(per, 1e-6))))
    t0 = time.perf_counter()
    out = oracle.md_run(box.x, box.v, box.box, tabs, steps, **kw)
    dt = time.perf_counter() - t0
    assert out["code"] == 0
    # the same oracle on one thread (bitwise the same results), a shorter sample
    oracle.set_threads(1)
    try:
        s1 = max(3, steps // (4 * max(threads, 1)))
        t0 = time.perf_counter()
        out1 = oracle.md_run(box.x, box.v, box.box, tabs, s1, **kw)
        dt1 = time.perf_counter() - t0
    finally:
        oracle.set_threads(threads)
    assert out1["code"] == 0
    return dict(value=steps / dt, unit="timesteps/s", cores=threads, kind="oracle",
                sample=f"{steps} velocity-Verlet steps of the same {box.n}-atom float64 workload "
                       f"(first list build included), OpenMP over atoms",
                atom_steps_per_s=steps * box.n / dt, cpu_model=_cpu_model(),
                single_thread={"value": s1 / dt1, "unit": "timesteps/s", "steps": s1})


def cpu_c1(tabs):
    """The oracle on the 2,000-atom workload: all of its 100 steps."""
    import oracle
    from workloads import configs, potential

    box = configs.config_small()
    t0 = time.perf_counter()
    out = oracle.md_run(box.x, box.v, box.box, tabs, 100, mass=configs.MASS, dt=configs.DT,
                        r_cut=potential.RC, skin=configs.SKIN, ftm2v=configs.FTM2V)
    dt = time.perf_counter() - t0
    assert out["code"] == 0
    return {"steps": 100, "timesteps_per_s": round(100 / dt, 2),
            "atom_steps_per_s": round(100 * box.n / dt, 1), "cores": oracle.get_threads()}


def cpu_c3(tabs, big, snaps):
    """The oracle on the 802,344-atom workload: 10 velocity-Verlet steps (rate),
    and its forces on the mixed run's positions at each snapshot, where the
    mixed and the float64 GPU forces are compared with it."""
    import oracle
    from workloads import configs, potential

    t0 = time.perf_counter()
    out = oracle.md_run(big.x, big.v, big.box, tabs, 10, mass=configs.MASS, dt=configs.DT,
                        r_cut=potential.RC, skin=configs.SKIN, ftm2v=configs.FTM2V)
    dt = time.perf_counter() - t0
    assert out["code"] == 0
    rows = []
    t_eval = 0.0
    for sn in snaps:
        t0 = time.perf_counter()
        ref = oracle.forces_at(sn["x"], big.box, tabs, potential.RC, configs.SKIN)
        t_eval += time.perf_counter() - t0
        fr = ref["f"]
        rms_f = float(np.sqrt(np.mean(np.sum(fr * fr, axis=1))))
        em = np.linalg.norm(sn["f_mixed"] - fr, axis=1)
        e64 = np.linalg.norm(sn["f_fp64"] - fr, axis=1)
        rows.append({"step": sn["step"], "force_rms_eVA": rms_f,
                     "mixed_max_eVA": float(em.max()),
                     "mixed_rms_eVA": float(np.sqrt(np.mean(em * em))),
                     "mixed_max_rel_to_rms_force": float(em.max() / rms_f),
                     "fp64_gpu_max_eVA": float(e64.max()),
                     "fp64_gpu_max_rel_to_max_force": float(e64.max()
                                                            / np.linalg.norm(fr, axis=1).max())})
    return {"oracle_steps": 10, "oracle_timesteps_per_s": round(10 / dt, 3),
            "oracle_atom_steps_per_s": round(10 * big.n / dt, 1),
            "oracle_snapshot_force_evaluations": len(snaps),
            "oracle_s_per_force_evaluation": round(t_eval / max(len(snaps), 1), 3),
            "cores": oracle.get_threads(), "force_error_vs_oracle": rows}


def cpu_c5(problem):
    """The oracle's force-matching loss and reverse-mode gradient over the same
    64 configurations: one gradient evaluation, timed."""
    import oracle

    t0 = time.perf_counter()
    loss, _, _ = oracle.fm_loss_grad(problem["x"], problem["offsets"], problem["boxes"],
                                     problem["tabs"], problem["fref"])
    dt = time.perf_counter() - t0
    return {"gradient_evaluations_per_s": round(1.0 / dt, 3), "s_per_gradient_evaluation":
            round(dt, 4), "loss": loss, "cores": oracle.get_threads()}


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


WORKLOADS = {
    "128k": "EAM BCC 40x40x40 cells (128,000 atoms), a=3.304 A, 300 K, skin 0.3 A, dt 1 fs, "
            "NVE, float64",
    "810k": "EAM BCC 74x74x74 cells minus 1% vacancies (802,344 atoms), a=3.304 A, 2,500 K, "
            "skin 0.3 A, dt 1 fs, NVE, float64",
}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--sections", default=",".join(SECTIONS),
                    help="comma-separated secondary workloads to run")
    ap.add_argument("--secondary-steps", type=int, default=5000)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--lpa", type=int, default=0)
    ap.add_argument("--c1-graph-only", action="store_true",
                    help="c1 without its persistent-launch comparison (for rocprofv3 runs)")
    ap.add_argument("--c1-lpa", type=int, default=0,
                    help="c1's lanes per atom (0: the autotuner's pick, whose timings under "
                         "rocprofv3 differ from a plain run)")
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--sequential-steps", type=int, default=20)
    ap.add_argument("--copy-probe-mib", type=int, default=512,
                    help="size of the plain device copy that measures achievable HBM bandwidth")
    ap.add_argument("--workload", choices=("128k", "810k"), default="128k",
                    help="the timed workload (810k: for profiling at the paper's scale; the "
                         "reported metric is the 128k one)")
    ap.add_argument("--fm-only", action="store_true",
                    help="time only the force-matching gradient (one JSON object, for profiling)")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the EAM path here is built and timed on a "
              "single MI355X (multi-GPU sharding is design-only); run with --gpus 1.",
              file=sys.stderr)
        return 2

    import torch

    from paper_2405_07898_amd import md
    from workloads import configs, potential

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    md.lib()
    tabs = potential.md_tables()
    if args.fm_only:
        res, _ = bench_fm(torch, md, configs, potential, tabs)
        print(json.dumps({"force_matching": res}), flush=True)
        return 0
    copy = copy_probe(torch, args.copy_probe_mib) if args.copy_probe_mib > 0 else None
    if copy:
        log(f"copy probe: {copy}")
    out, box = bench_headline(torch, md, configs, tabs, args, copy["gbs"] if copy else None)
    if copy:
        out["copy_probe"] = copy
    sections = set() if args.no_secondary else set(args.sections.split(","))
    big, snaps, fm_problem = None, [], None
    if "c1" in sections:
        out["c1_2000"] = bench_c1(torch, md, configs, tabs, persistent=not args.c1_graph_only,
                                  lpa=args.c1_lpa)
        log(f"  c1: {out['c1_2000']}")
    if "c2" in sections:
        out["c2_10000"] = bench_c2_series(torch, md, configs, tabs)
        log(f"  c2: {({k: v for k, v in out['c2_10000'].items() if k != 'series'})}")
    if "c3" in sections:
        out["c3_810k"], big, snaps = bench_c3(torch, md, configs, tabs, args)
    if "slab" in sections:
        log("slab 801,792 atoms")
        out["slab_801792"] = bench_slab(torch, md, configs, tabs, args.secondary_steps)
        log(f"  slab: {out['slab_801792']}")
    if "half" in sections:
        out["half_list_128k"] = bench_half(torch, md, configs, tabs, 5000)
        log(f"  half list: {out['half_list_128k']}")
    if "alloy" in sections:
        out["alloy_128k"] = bench_alloy(torch, md, configs, potential, 5000)
        log(f"  binary alloy: {out['alloy_128k']}")
    if "perf_model" in sections:
        out["perf_model"] = perf_model(torch, md, configs, tabs)
        pm = out["perf_model"]
        log(f"  perf model: every step {pm['every_step']}; list reuse {pm['list_reuse']}")
    if "batched" in sections:
        out["batched_256"] = bench_batched(torch, md, configs, tabs, args)
        log(f"  batched: {out['batched_256']}")
    if "fm" in sections:
        out["force_matching"], fm_problem = bench_fm(torch, md, configs, potential, tabs)
        log(f"  force matching: {out['force_matching']}")

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(box, tabs)
        log(f"  {out['cpu_baseline']}")
        if "c1" in sections:
            out["cpu_baseline"]["c1_2000"] = cpu_c1(tabs)
        if snaps:
            c3 = cpu_c3(tabs, big, snaps)
            out["c3_810k"]["force_error_vs_oracle"] = c3.pop("force_error_vs_oracle")
            out["cpu_baseline"]["c3_810k"] = c3
        if fm_problem is not None:
            out["cpu_baseline"]["c5_force_matching"] = cpu_c5(fm_problem)
        log(f"  {out['cpu_baseline']}")

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
