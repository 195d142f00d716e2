"""Benchmark of the EAM timestep loop on one MI355X.

Default workload: 128,000-atom BCC box (40^3 cells, a = 3.304 A), float64,
300 K, skin 0.3 A, dt = 1 fs, hipGraph chunks of 100 steps; K timed steps
after W warm-up steps.  Prints one JSON line (metric: timesteps/s, plus
atom-steps/s, roofline of the dominant kernel, CPU-oracle baseline and the
810,448-site float64 / mixed-precision secondary points).

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
KERNEL_SRC = os.path.join(ROOT, "paper_2405_07898_amd", "csrc", "md_kernels.hip")
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "force_integrate_128k_traffic.json")
# re-sort atoms by cell every 2 graph chunks (200 steps): the specified potential's
# lattice melts and its atoms diffuse, so the cell order of the slots decays
# (measured at 128,000 atoms: 55.6 us/step re-sorting every 2 chunks against
# 59.9 every 10)
SORT_EVERY = 2


def log(msg: str) -> None:
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def force_pass_bytes(n_atoms: int, n_l: float, mixed: bool) -> float:
    """Algorithmic HBM bytes of one force+integrate launch.

    Per atom: x (24) + F' (8, 4 mixed) + list length (4) + list entries (4 n_l)
    + v read and write (48) + new x (24) + x_ref (24); neighbour gathers are
    cache-served and not counted.
    """
    per = 24 + (4 if mixed else 8) + 4 + 4 * n_l + 48 + 24 + 24
    return n_atoms * per


def force_pass_flops(n_atoms: int, n_l: float, n_int: float) -> float:
    """Algorithmic flops (paper Table "flopmodel"): 9 per list entry (distance and
    test), 31 per interaction (r^-1, r, segment, rho' and phi', force), 8 per atom
    (F' sum reuse and the Verlet update)."""
    return n_atoms * (9 * n_l + 31 * n_int + 8)


def source_hash() -> str:
    with open(KERNEL_SRC, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()


def load_traffic(n_launch_atoms: int):
    """HBM traffic per launch from committed rocprofv3 counter runs, if they
    were taken on the current kernel source."""
    if not os.path.exists(TRAFFIC_FILE):
        return None
    with open(TRAFFIC_FILE) as f:
        t = json.load(f)
    if t.get("kernel_source_sha256") != source_hash() or t.get("n_atoms") != n_launch_atoms:
        return None
    return t.get("bytes_per_launch")


def make_system(md, box, tabs, *, precision, chunk, lpa=0):
    from workloads import configs, potential

    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=configs.SKIN,
                       ftm2v=configs.FTM2V, precision=precision, chunk_steps=chunk,
                       lanes_per_atom=lpa, nbr_capacity=128, cell_capacity=64, sort_every=SORT_EVERY)
    s = md.System(p, tabs, [box.n], box.box[None, :])
    s.set_state(box.x, box.v)
    s.build_neighbors()
    return s


def time_steps(torch, s, steps: int) -> float:
    """Seconds for `steps` MD steps, bracketed by stream events and syncs."""
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
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


def copy_probe(torch, mib: int, reps: int = 5) -> dict:
    """A plain elementwise copy (y = -x, float64) of known size: it reads and
    writes mib MiB once per launch, so hardware byte counters read on it give
    the factor between counter units and bytes moved."""
    n = mib * (1 << 20) // 8
    src = torch.rand(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        torch.neg(src, out=dst)
    e1.record()
    torch.cuda.synchronize()
    us = e0.elapsed_time(e1) * 1e3 / reps
    return {"bytes_read": n * 8, "bytes_written": n * 8, "launches": reps,
            "avg_us": round(us, 2), "gbs": round(2 * n * 8 / (us * 1e-6) / 1e9, 1)}


def cpu_baseline(box, tabs, budget_s: float = 15.0):
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


def _cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def bench_small(torch, md, configs, tabs):
    """2,000-atom box, 100-step chunks (launch-latency regime): a captured graph
    per chunk, and for comparison one persistent cooperative launch per chunk."""
    from workloads import potential

    box = configs.config_small()
    s = make_system(md, box, tabs, precision=md.MD_FP64, chunk=100)
    lpa, _ = s.autotune(50)
    s.step(100)
    sec, _ = time_steps(torch, s, 2000)
    st = s.stats()
    s.close()
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=configs.SKIN,
                       ftm2v=configs.FTM2V, precision=md.MD_FP64, chunk_steps=100,
                       lanes_per_atom=8, nbr_capacity=128, cell_capacity=64,
                       sort_every=SORT_EVERY, launch_mode=md.MD_LAUNCH_PERSISTENT)
    sp = md.System(p, tabs, [box.n], box.box[None, :])
    sp.set_state(box.x, box.v)
    sp.build_neighbors()
    sp.step(100)
    sec_p, _ = time_steps(torch, sp, 2000)
    sp.close()
    return {"n_atoms": box.n, "steps": 2000, "timesteps_per_s": round(2000 / sec, 1),
            "atom_steps_per_s": round(2000 / sec * box.n, 1), "lanes_per_atom": lpa,
            "rebuilds": st["rebuilds"],
            "persistent_launch_timesteps_per_s": round(2000 / sec_p, 1)}


def bench_slab(torch, md, configs, tabs, steps):
    """The paper's benchmark geometry (Sec. IV-B): an 801,792-atom BCC slab of
    256 x 261 x 6 cells, open in x and y, periodic through its thickness, at
    300 K, with the specified potential."""
    box = configs.config_slab_801792()
    s = make_system(md, box, tabs, precision=md.MD_FP64, chunk=100)
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
    from workloads import potential

    box = configs.config_128k()
    out = {"n_atoms": box.n, "steps": steps}
    for name, mode in (("full", md.MD_LIST_FULL), ("half", md.MD_LIST_HALF)):
        p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=configs.SKIN,
                           ftm2v=configs.FTM2V, precision=md.MD_FP64, chunk_steps=100,
                           nbr_capacity=128, cell_capacity=64, sort_every=SORT_EVERY,
                           list_mode=mode)
        s = md.System(p, tabs, [box.n], box.box[None, :])
        s.set_state(box.x, box.v)
        s.build_neighbors()
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
    p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC, skin=configs.SKIN,
                       ftm2v=configs.FTM2V, precision=md.MD_FP64, chunk_steps=100,
                       nbr_capacity=128, cell_capacity=64, sort_every=SORT_EVERY, n_types=2)
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


def perf_model(torch, md, configs, tabs, steps: int = 1000):
    """Linear model of the step time at fixed N, t = A n_l + B n_int + C (the
    paper's Eq. linearmodel / Table "regression", with list entries standing
    in for candidates): dt = 0 sweeps over the interaction cutoff and the skin
    on the 128,000-atom lattice, so the list never changes."""
    from workloads import potential

    box = configs.config_128k()
    rows = []
    for rc in (3.0, 3.5, 4.0, 5.0):
        for skin in (0.3, 0.8, 1.4, 2.2):
            p = md.make_params(mass=configs.MASS, dt=0.0, r_cut=rc, skin=skin,
                               ftm2v=configs.FTM2V, precision=md.MD_FP64, chunk_steps=100,
                               lanes_per_atom=2, nbr_capacity=160, cell_capacity=64,
                               sort_every=0)
            s = md.System(p, tabs, [box.n], box.box[None, :])
            s.set_state(box.x, box.v)
            s.build_neighbors()
            s.step(200)
            sec, _ = time_steps(torch, s, steps)
            n_l = s.stats()["list_entries"] / box.n
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
            rows.append((n_l, n_int / len(pick), sec / steps * 1e6, rc, skin))
    m = np.array(rows)
    X = np.column_stack([m[:, 0], m[:, 1], np.ones(len(m))])
    coef, *_ = np.linalg.lstsq(X, m[:, 2], rcond=None)
    pred = X @ coef
    r2 = 1.0 - np.sum((m[:, 2] - pred) ** 2) / np.sum((m[:, 2] - m[:, 2].mean()) ** 2)
    return {"n_atoms": box.n, "steps_per_point": steps, "lanes_per_atom": 2,
            "us_per_step_per_list_entry": round(float(coef[0]), 4),
            "us_per_step_per_interaction": round(float(coef[1]), 4),
            "us_per_step_fixed": round(float(coef[2]), 3),
            "ns_per_atom_list_entry": round(float(coef[0]) * 1e3 / box.n, 6),
            "ns_per_atom_interaction": round(float(coef[1]) * 1e3 / box.n, 6),
            "r2": round(float(r2), 5),
            "points": [{"r_cut": r[3], "skin": r[4], "n_l": round(r[0], 3),
                        "n_int": round(r[1], 3), "us_per_step": round(r[2], 3)} for r in rows]}


def bench_batched(torch, md, configs, tabs, args):
    """256 replicas (5-20 cells, 0-2 % vacancies, 300-2000 K) in one launch per pass,
    against a sequential loop of single-replica contexts."""
    from workloads import potential

    reps = configs.config_batch(256)
    n_tot = sum(b.n for b in reps)
    res = {"n_replicas": len(reps), "n_atoms_total": n_tot}
    for name, prec in (("fp64", md.MD_FP64), ("mixed", md.MD_MIXED)):
        p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC,
                           skin=configs.SKIN, ftm2v=configs.FTM2V, precision=prec,
                           chunk_steps=100, nbr_capacity=128, cell_capacity=64)
        s = md.System(p, tabs, [b.n for b in reps], np.stack([b.box for b in reps]))
        s.set_state(np.concatenate([b.x for b in reps]), np.concatenate([b.v for b in reps]))
        s.build_neighbors()
        lpa, _ = s.autotune(20)
        s.step(100)
        steps = args.batched_steps
        sec, _ = time_steps(torch, s, steps)
        s.close()
        res[name] = {"steps": steps, "lanes_per_atom": lpa,
                     "timesteps_per_s": round(steps / sec, 2),
                     "atom_steps_per_s": round(steps * n_tot / sec, 1)}
    # sequential per-replica loop (float64), same kernels, one context per replica
    seq_steps = args.sequential_steps
    systems = []
    for b in reps:
        p = md.make_params(mass=configs.MASS, dt=configs.DT, r_cut=potential.RC,
                           skin=configs.SKIN, ftm2v=configs.FTM2V, chunk_steps=50,
                           nbr_capacity=128, cell_capacity=64)
        s = md.System(p, tabs, [b.n], b.box[None, :])
        s.set_state(b.x, b.v)
        s.build_neighbors()
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
    sec = time.perf_counter() - t0
    prob.close()
    return {"n_configs": 64, "n_atoms_total": int(x.shape[0]),
            "gradient_evaluations_per_s": round(reps / sec, 2),
            "ms_per_gradient_evaluation": round(sec / reps * 1e3, 4)}


WORKLOADS = {
    "128k": "EAM BCC 40x40x40 cells (128,000 atoms), a=3.304 A, 300 K, skin 0.3 A, dt 1 fs, "
            "NVE, float64, hipGraph chunks of 100 steps",
    "810k": "EAM BCC 74x74x74 cells minus 1% vacancies (802,344 atoms), a=3.304 A, 2,500 K, "
            "skin 0.3 A, dt 1 fs, NVE, float64, hipGraph chunks of 100 steps",
}


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10000)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-secondary", action="store_true")
    ap.add_argument("--secondary-steps", type=int, default=5000)
    ap.add_argument("--kernel-reps", type=int, default=200)
    ap.add_argument("--lpa", type=int, default=0)
    ap.add_argument("--batched-steps", type=int, default=1000)
    ap.add_argument("--sequential-steps", type=int, default=20)
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="also run a plain device copy of this many MiB (calibrates HBM counters)")
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
        print(json.dumps({"force_matching": bench_fm(torch, md, configs, potential, tabs)}),
              flush=True)
        return 0
    box = configs.config_128k() if args.workload == "128k" else configs.config_810k()
    log(f"workload {args.workload}: n={box.n} box={box.box[0]:.3f} A; building")
    s = make_system(md, box, tabs, precision=md.MD_FP64, chunk=100, lpa=args.lpa)
    if args.lpa == 0:
        lpa, us = s.autotune(50)
        log(f"autotune: {lpa} lanes per atom ({us:.1f} us per density+force)")
    pe0, ke0 = s.energy()
    log(f"warmup {args.warmup} steps")
    s.step(args.warmup)
    st0 = s.stats()
    log(f"timing {args.steps} steps")
    sec, wall = time_steps(torch, s, args.steps)
    st1 = s.stats()
    pe1, ke1 = s.energy()
    ts = args.steps / sec
    n_l = st1["list_entries"] / box.n
    log(f"{ts:.1f} timesteps/s ({sec * 1e3 / args.steps:.4f} ms/step, wall {wall:.3f} s), "
        f"rebuilds {st1['rebuilds'] - st0['rebuilds']}, mean list {n_l:.2f}")

    # dominant kernel: force + integrate, timed per launch on the library stream
    dens_us = time_kernel(torch, s, md, md.PASS_DENSITY, args.kernel_reps)
    force_us = time_kernel(torch, s, md, md.PASS_FORCE_RAW, args.kernel_reps)
    byts = force_pass_bytes(box.n, n_l, False)
    flops = force_pass_flops(box.n, n_l, n_l)
    gbs = byts / (force_us * 1e-6) / 1e9
    tfl = flops / (force_us * 1e-6) / 1e12
    # the roofline that binds: intensity below the float64 ridge -> HBM
    ridge = FP64_PEAK_TFLOPS * 1e12 / (HBM_PEAK_GBS * 1e9)
    bound = "hbm" if flops / byts < ridge else "alu"
    traffic = load_traffic(box.n)
    roof = {"bound": bound, "kernel": "k_force_integrate<fp64>",
            "achieved": round(gbs, 1) if bound == "hbm" else round(tfl, 3),
            "peak": HBM_PEAK_GBS if bound == "hbm" else FP64_PEAK_TFLOPS,
            "unit": "GB/s" if bound == "hbm" else "TFLOP/s",
            "frac": round((gbs / HBM_PEAK_GBS) if bound == "hbm" else (tfl / FP64_PEAK_TFLOPS), 4),
            "traffic": traffic,
            "algorithmic_bytes_per_launch": byts, "algorithmic_flops_per_launch": flops,
            "avg_kernel_us": round(force_us, 3),
            "alu_frac": round(tfl / FP64_PEAK_TFLOPS, 4), "mean_list_length": round(n_l, 3),
            "density_kernel_us": round(dens_us, 3)}
    log(f"force pass {force_us:.2f} us -> {gbs:.0f} GB/s ({roof['frac'] * 100:.1f}% HBM), "
        f"{tfl:.2f} TFLOP/s; density {dens_us:.2f} us")
    s.close()

    out = {
        "metric": METRIC, "value": round(ts, 2), "unit": "timesteps/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(sec * 1e3 / args.steps, 5), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "f64", "data": "synthetic",
        "config": {"workload": WORKLOADS[args.workload],
                   "n_atoms": box.n, "chunk_steps": 100},
        "atom_steps_per_s": round(ts * box.n, 1),
        "energy_drift_per_atom_eV": float(abs((pe1[0] + ke1[0]) - (pe0[0] + ke0[0])) / box.n),
        "rebuilds_in_timed_region": int(st1["rebuilds"] - st0["rebuilds"]),
        "wall_s_timed": round(wall, 4),
        "roofline": roof,
    }

    if not args.no_secondary:
        big = configs.config_810k()
        sec_out = {}
        for name, prec in (("fp64", md.MD_FP64), ("mixed", md.MD_MIXED)):
            log(f"secondary 810k {name}: n={big.n}")
            sb = make_system(md, big, tabs, precision=prec, chunk=100, lpa=args.lpa)
            if args.lpa == 0:
                lpa, us = sb.autotune(20)
                log(f"  autotune: {lpa} lanes per atom ({us:.1f} us per density+force)")
            sb.step(100)
            t2, _ = time_steps(torch, sb, args.secondary_steps)
            stb = sb.stats()
            nlb = stb["list_entries"] / big.n
            fu = time_kernel(torch, sb, md, md.PASS_FORCE_RAW, 50)
            b2 = force_pass_bytes(big.n, nlb, prec == md.MD_MIXED)
            sec_out[name] = {"timesteps_per_s": round(args.secondary_steps / t2, 2),
                             "atom_steps_per_s": round(args.secondary_steps / t2 * big.n, 1),
                             "force_pass_us": round(fu, 3),
                             "force_pass_hbm_frac": round(b2 / (fu * 1e-6) / 1e9 / HBM_PEAK_GBS, 4),
                             "mean_list_length": round(nlb, 3), "rebuilds": stb["rebuilds"]}
            if name == "fp64":
                f64, _, _ = sb.compute_forces()
                x64, _, _ = sb.get_state(want_f=False)
            else:
                # mixed forces at the float64 run's positions, against its float64 forces
                sb.set_state(x64, torch.zeros_like(x64))
                sb.build_neighbors()
                fm, _, _ = sb.compute_forces()
                err = (fm - f64).norm(dim=1)
                rms = f64.norm(dim=1).pow(2).mean().sqrt().item()
                sec_out[name]["force_err_vs_fp64_max_eVA"] = err.max().item()
                sec_out[name]["force_err_vs_fp64_rms_eVA"] = err.pow(2).mean().sqrt().item()
                sec_out[name]["force_rms_eVA"] = rms
            sb.close()
            log(f"  {sec_out[name]}")
        out["secondary_810k"] = {"n_atoms": big.n, "steps": args.secondary_steps,
                                 "workload": "74^3 BCC sites - 1% vacancies, 2500 K", **sec_out}

    if not args.no_secondary:
        log("secondary slab 801,792 atoms")
        out["secondary_slab_801792"] = bench_slab(torch, md, configs, tabs, args.secondary_steps)
        log(f"  slab: {out['secondary_slab_801792']}")
        out["secondary_half_list_128k"] = bench_half(torch, md, configs, tabs, 5000)
        log(f"  half list: {out['secondary_half_list_128k']}")
        out["secondary_alloy_128k"] = bench_alloy(torch, md, configs, potential, 5000)
        log(f"  binary alloy: {out['secondary_alloy_128k']}")
        out["secondary_small_2000"] = bench_small(torch, md, configs, tabs)
        out["secondary_perf_model"] = perf_model(torch, md, configs, tabs)
        pm = out["secondary_perf_model"]
        log(f"  perf model: t = {pm['us_per_step_per_list_entry']} n_l + "
            f"{pm['us_per_step_per_interaction']} n_int + {pm['us_per_step_fixed']} us, "
            f"r2 {pm['r2']}")
        log(f"  small: {out['secondary_small_2000']}")
        out["secondary_batched_256"] = bench_batched(torch, md, configs, tabs, args)
        log(f"  batched: {out['secondary_batched_256']}")
        out["secondary_force_matching"] = bench_fm(torch, md, configs, potential, tabs)
        log(f"  force matching: {out['secondary_force_matching']}")

    if args.copy_probe_mib > 0:
        out["copy_probe"] = copy_probe(torch, args.copy_probe_mib)
        log(f"copy probe: {out['copy_probe']}")

    if not args.no_cpu_baseline:
        log("cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(box, tabs)
        log(f"  {out['cpu_baseline']}")

    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
