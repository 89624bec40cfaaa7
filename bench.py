"""Benchmark of the HIP spectral Cahn-Hilliard stepper on one MI355X.

A step is one pass of the whole per-step hot path (inverse y, fused x with f', forward y, fused z
with the k-space update) over the seeded synthetic field, which is resident in HBM before the
timed region starts.  The default workload is the 1024^3 periodic quench (mean 0, amplitude 0.05,
seed 3, dt 0.5, spectral wavenumbers).  The line also carries:
  roofline     - the dominant kernel's algorithmic bytes per launch over its average launch
                 duration, timed with HIP events on the launch stream inside the timed region;
  cpu_baseline - the FP64 oracle (SciPy FFTs) timed on this host on a bounded sample;
  extra        - smaller and zero-flux grids, the exponential (ETD1) stepper and the Allen-Cahn
                 model on the same workload, Dirichlet boundaries, the Gray-Scott model, the
                 inverse-problem gradient and the learned coarse stepper.

usage: python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload NAME] [--no-cpu-baseline]
       python bench.py --summarize-profile DIR [--workload NAME]
The second form turns the three rocprofv3 runs listed in PROFILE_COMMANDS (kernel trace, then
FETCH_SIZE, then WRITE_SIZE, each writing under DIR) into profiles/kernels_<workload>.md and
profiles/traffic_<workload>.json.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
PASS_NAMES = ["y_inverse", "x_fused_fprime", "y_forward", "z_fused_update"]
PROFILES = os.path.join(ROOT, "profiles")


def kernel_source_hash() -> str:
    """Hash of the HIP sources the Cahn-Hilliard step is built from (all but the surrogate's
    evx_net.hip); counter-based traffic figures are used only while it matches."""
    import hashlib
    csrc = os.path.join(ROOT, "paper_2507_21748_amd", "csrc")
    h = hashlib.sha256()
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".hpp", ".hip")) and name != "evx_net.hip":
            h.update(name.encode())
            h.update(open(os.path.join(csrc, name), "rb").read())
    return h.hexdigest()[:16]


def measured_traffic(workload: str, kernel: str):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 FETCH_SIZE / WRITE_SIZE
    summary (scaled by the copy-kernel calibration), or None if absent or stale."""
    path = os.path.join(PROFILES, f"traffic_{workload}.json")
    if not os.path.exists(path):
        return None
    rec = json.load(open(path))
    if rec.get("source_hash") != kernel_source_hash():
        return None
    k = rec.get("kernels", {}).get(kernel)
    return None if k is None else k["bytes_per_launch"]


# The rocprofv3 runs summarized by --summarize-profile (run from /tmp with TMPDIR=/tmp; {d} is
# the output directory, {w} the workload).  Counters are taken in runs of their own.
PROFILE_COMMANDS = [
    ("kt", "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv -d {d}/kt -o kt "
           "-- python3 {root}/bench.py --workload {w} --steps 20 --warmup 2 --no-cpu-baseline "
           "--no-extra"),
    ("fs", "timeout -s KILL 240 rocprofv3 --pmc FETCH_SIZE --output-format csv -d {d}/fs -o fs "
           "-- python3 {root}/bench.py --workload {w} --steps 4 --warmup 1 --no-cpu-baseline "
           "--no-extra"),
    ("ws", "timeout -s KILL 240 rocprofv3 --pmc WRITE_SIZE --output-format csv -d {d}/ws -o ws "
           "-- python3 {root}/bench.py --workload {w} --steps 4 --warmup 1 --no-cpu-baseline "
           "--no-extra"),
]


# Kernel-trace runs of single extras, summarized by --summarize-trace into
# profiles/kernels_<name>.md (same conventions as PROFILE_COMMANDS).
TRACE_COMMANDS = {
    "surrogate512": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv "
                    "-d {d}/kt -o kt -- python3 {root}/bench.py --extra-only surrogate512",
    "inverse128": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv "
                  "-d {d}/kt -o kt -- python3 {root}/bench.py --extra-only inverse128",
    "varmob256": "timeout -k 10 300 rocprofv3 --kernel-trace --stats --output-format csv "
                 "-d {d}/kt -o kt -- python3 {root}/bench.py --extra-only varmob256",
}


def summarize_trace(d: str, name: str):
    """profiles/kernels_<name>.md from the --stats CSV of the TRACE_COMMANDS run under d."""
    import csv
    import glob
    stats = list(csv.DictReader(open(glob.glob(os.path.join(d, "kt", "*kernel_stats.csv"))[0])))
    cmd = TRACE_COMMANDS[name].format(d="$OUT", root="$REPO")
    lines = [f"# rocprofv3 kernel trace: {name}", "",
             "Command (REPO = repository root, OUT = an output directory; run from /tmp with "
             f"TMPDIR=/tmp), then `python bench.py --summarize-trace $OUT --workload {name}`:", "",
             f"    {cmd}", "", "| kernel | calls | avg us | total ms | % time |", "|---|---|---|---|---|"]
    for r in stats[:20]:
        lines.append(f"| `{r['Name'][:90]}` | {r['Calls']} | {float(r['AverageNs']) * 1e-3:.1f} | "
                     f"{float(r['TotalDurationNs']) * 1e-6:.3f} | {float(r['Percentage']):.1f} |")
    os.makedirs(PROFILES, exist_ok=True)
    open(os.path.join(PROFILES, f"kernels_{name}.md"), "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def _pass_of_kernel(name: str):
    """Pass of a stepper kernel from its template arguments (col_kernel<N, BC, MODE>: MODE 0 forward
    y, 1 inverse y, 3 fused z update; row_kernel<NH, BC, MODE>: MODE 0 fused x with f')."""
    import re
    m = re.search(r"evx::(col|row)_kernel<(\d+), (\d+), (\d+)>", name)
    if not m:
        return None
    kind, mode = m.group(1), int(m.group(4))
    if kind == "col":
        return {0: "y_forward", 1: "y_inverse", 3: "z_fused_update"}.get(mode)
    return "x_fused_fprime" if mode == 0 else None


def summarize_profile(d: str, workload: str):
    """Kernel-trace statistics and calibrated HBM traffic per pass from the rocprofv3 CSVs."""
    import csv
    import glob
    from paper_2507_21748_amd.inputs import WORKLOADS
    w = WORKLOADS[workload]
    nbytes = dict(zip(PASS_NAMES, pass_bytes(w.shape, w.bc)))
    stats = list(csv.DictReader(open(glob.glob(os.path.join(d, "kt", "*kernel_stats.csv"))[0])))

    def counters(sub):
        rows = csv.DictReader(open(glob.glob(os.path.join(d, sub, "*counter_collection.csv"))[0]))
        per = {}
        for r in rows:
            per.setdefault(r["Kernel_Name"], []).append(float(r["Counter_Value"]) * 1024.0)
        return per

    fetch, write = counters("fs"), counters("ws")
    # calibration: the probe's device-to-device copy of a known size (copy_probe, 2 GiB each way)
    copy = [k for k in fetch if "copyBuffer" in k][0]
    known = float(2 << 30)
    big_f = [v for v in fetch[copy] if v > known / 8]
    big_w = [v for v in write[copy] if v > known / 8]
    f_scale = known / (sum(big_f) / len(big_f))
    w_scale = known / (sum(big_w) / len(big_w))
    by_pass = {}
    for name in fetch:
        p = _pass_of_kernel(name)
        if p is None:
            continue
        f = sum(fetch[name]) / len(fetch[name]) * f_scale
        wr = sum(write[name]) / len(write[name]) * w_scale
        by_pass[p] = {"kernel": name, "fetch_bytes": f, "write_bytes": wr,
                      "bytes_per_launch": f + wr,
                      "algorithmic_bytes": nbytes[p], "ratio": (f + wr) / nbytes[p]}
    cmds = [c.format(d="$OUT", w=workload, root="$REPO") for _, c in PROFILE_COMMANDS]
    src = kernel_source_hash()
    rec = {"workload": workload, "source_hash": src, "fetch_scale": f_scale,
           "write_scale": w_scale, "commands": cmds, "kernels": by_pass}
    os.makedirs(PROFILES, exist_ok=True)
    json.dump(rec, open(os.path.join(PROFILES, f"traffic_{workload}.json"), "w"), indent=1)
    lines = [f"# rocprofv3 summary: {workload}", "",
             f"Grid {'x'.join(map(str, w.shape[::-1]))}, {w.bc}, {w.scheme}; kernel source "
             f"hash {src}.", "", "Commands (REPO = repository root, OUT = an output directory; run "
             "from /tmp with TMPDIR=/tmp), then "
             f"`python bench.py --summarize-profile $OUT --workload {workload}`:", ""]
    lines += [f"    {c}" for c in cmds]
    lines += ["", "## Kernel trace (--stats)", "",
              "| kernel | pass | calls | avg ms | % time | algorithmic GB/s |",
              "|---|---|---|---|---|---|"]
    for r in stats[:12]:
        p = _pass_of_kernel(r["Name"])
        avg = float(r["AverageNs"]) * 1e-6
        gbs = f"{nbytes[p] / (avg * 1e-3) / 1e9:.0f}" if p else ""
        lines.append(f"| `{r['Name'][:70]}` | {p or ''} | {r['Calls']} | {avg:.4f} | "
                     f"{r['Percentage']} | {gbs} |")
    lines += ["", "## HBM traffic per launch (FETCH_SIZE, WRITE_SIZE)", "",
              f"Calibration on a 2 GiB device copy: FETCH_SIZE x {f_scale:.4f}, "
              f"WRITE_SIZE x {w_scale:.4f}.", "",
              "| pass | read GB | written GB | total GB | algorithmic GB | ratio |",
              "|---|---|---|---|---|---|"]
    for p in PASS_NAMES:
        if p in by_pass:
            b = by_pass[p]
            lines.append(f"| {p} | {b['fetch_bytes'] / 1e9:.3f} | {b['write_bytes'] / 1e9:.3f} | "
                         f"{b['bytes_per_launch'] / 1e9:.3f} | {b['algorithmic_bytes'] / 1e9:.3f}"
                         f" | {b['ratio']:.3f} |")
    open(os.path.join(PROFILES, f"kernels_{workload}.md"), "w").write("\n".join(lines) + "\n")
    print("\n".join(lines))


def copy_probe(torch, gib: float, reps: int = 3):
    """A plain device-to-device copy of a known size (torch's copy kernel), for calibrating the
    FETCH_SIZE / WRITE_SIZE counters and as a measured bandwidth ceiling."""
    n = int(gib * (1 << 30)) // 4
    a = torch.empty(n, dtype=torch.float32, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    b.copy_(a)
    torch.cuda.synchronize()
    # HIP events on the stream the copy runs on (torch's current stream)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        b.copy_(a)
    e1.record()
    e1.synchronize()
    secs = e0.elapsed_time(e1) / 1e3 / reps
    del a, b
    torch.cuda.empty_cache()
    return {"bytes_each_way": n * 4, "gbs": 2 * n * 4 / secs / 1e9, "timed_with": "hip events"}


def pass_bytes(shape, bc):
    """Algorithmic HBM bytes per launch of each pass: one read and one write of a spectral
    buffer (nz*ny*(nx/2+1) complex64, or nz*ny*nx float32 for zero flux); the z pass also reads
    and writes the state."""
    nz, ny, nx = shape
    spec = nz * ny * ((nx // 2 + 1) * 8 if bc == "periodic" else nx * 4)
    return [2 * spec, 2 * spec, 2 * spec, 4 * spec]


def run_workload(evx, torch, w, steps, warmup, timing=True, integrator=0, model=0, graph=None):
    from paper_2507_21748_amd.inputs import quench_field
    plan = evx.Plan(w.shape, w.bc, w.scheme, dx=w.dx)
    if graph is not None:
        plan.set_step_graph(graph)
    prm = evx.CHParams(dt=w.dt, M=w.M, kappa=w.kappa, A=w.A, integrator=integrator, model=model)
    c = torch.from_numpy(quench_field(w.shape, w.mean, w.amp, w.seed)).cuda()
    plan.begin(c)
    plan.advance(warmup, prm)
    torch.cuda.synchronize()
    plan.enable_pass_timing(timing)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.advance(steps, prm)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    plan.enable_pass_timing(False)
    ms, cnt = plan.read_pass_times() if timing else ([0] * 4, [0] * 4)
    plan.end(c)
    torch.cuda.synchronize()
    ok = bool(torch.isfinite(c).all().item())
    secs = t1 - t0
    vox = w.voxels
    out = {
        "voxel_steps_per_s": vox * steps / secs,
        "ms_per_step": 1e3 * secs / steps,
        "finite": ok,
        "workspace_bytes": plan.workspace_bytes,
    }
    if timing:
        nbytes = pass_bytes(w.shape, w.bc)
        per = {}
        for i, name in enumerate(PASS_NAMES):
            avg = ms[i] / max(cnt[i], 1)
            per[name] = {"avg_ms": avg, "launches": cnt[i],
                         "algorithmic_bytes": nbytes[i],
                         "gbs": nbytes[i] / (avg * 1e-3) / 1e9 if avg > 0 else None}
        out["passes"] = per
    del plan
    torch.cuda.empty_cache()
    return out


def adjoint_workload(evx, torch, w, steps: int = 200, every: int = 20):
    """The inverse-problem gradient: an nsteps rollout with spectral checkpoints every `every`
    steps (every = 0: every state recorded in the forward pass), then the backward sweep of
    hand-written adjoint steps (gradients for c0, kappa, M).  Returns wall times of the forward
    and backward halves."""
    from paper_2507_21748_amd.autograd import ch_rollout
    from paper_2507_21748_amd.inputs import quench_field
    plan = evx.Plan(w.shape, w.bc, w.scheme, dx=w.dx, ops=evx.OP_STEP | evx.OP_ADJOINT)
    c0 = torch.from_numpy(quench_field(w.shape, w.mean, w.amp, w.seed)).cuda().requires_grad_(True)
    kappa = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    M = torch.tensor(1.0, dtype=torch.float64, device="cuda", requires_grad=True)
    target = torch.zeros_like(c0)
    out = {}
    for rep in range(2):  # the first repetition warms up
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        cT = ch_rollout(c0, kappa, M, plan, steps, w.dt, w.A, every)
        loss = ((cT - target) ** 2).sum()
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        g = torch.autograd.grad(loss, (c0, kappa, M))
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        out = {"grid": list(w.shape[::-1]), "steps": steps, "checkpoint_every": every,
               "forward_ms": 1e3 * (t1 - t0), "backward_ms": 1e3 * (t2 - t1),
               "backward_ms_per_step": 1e3 * (t2 - t1) / steps,
               "finite": bool(all(torch.isfinite(x).all().item() for x in g))}
    del plan
    torch.cuda.empty_cache()
    return out


def gray_scott_workload(evx, torch, n: int = 256, steps: int = 100):
    """The Gray-Scott two-species model on a 256^3 periodic spectral grid (u ~ 1, v seeded as a
    0.25 +- 0.2 quench): ms per step (8 launches: reaction, 4 batched forward transforms, spectral
    update, 2 batched inverse transforms)."""
    from paper_2507_21748_amd.inputs import quench_field
    shape = (n, n, n)
    plan = evx.Plan(shape, "periodic", "spectral", ops=evx.OP_STEP | evx.OP_GRAY_SCOTT)
    u = torch.from_numpy(quench_field(shape, 0.75, 0.2, seed=11)).cuda()
    v = torch.from_numpy(quench_field(shape, 0.25, 0.2, seed=12)).cuda()
    prm = evx.GSParams(dt=1.0)
    plan.gs_step(u, v, 5, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.gs_step(u, v, steps, prm)
    torch.cuda.synchronize()
    secs = (time.perf_counter() - t0) / steps
    return {"grid": [n, n, n], "ms_per_step": 1e3 * secs,
            "finite": bool(torch.isfinite(u).all().item() and torch.isfinite(v).all().item())}


def varmob_workload(evx, torch, n: int = 256, steps: int = 100):
    """The variable-mobility Cahn-Hilliard step (M = D0 phi (1 - phi)) on a 256^3 periodic
    spectral grid, phi a 0.5 +- 0.2 quench: ms per step (the fused stencil pass, forward x and y,
    the z pass with the multiplier, inverse y, the inverse x pass that adds to phi)."""
    from paper_2507_21748_amd.inputs import quench_field
    shape = (n, n, n)
    plan = evx.Plan(shape, "periodic", "spectral", ops=evx.OP_STEP | evx.OP_VAR_MOBILITY)
    phi = torch.from_numpy(quench_field(shape, 0.5, 0.2, seed=13)).cuda()
    prm = evx.VMParams(dt=0.5, D0=1.0, gamma0=1.0, eps=2.0, M0=0.25)
    plan.vm_step(phi, 5, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.vm_step(phi, steps, prm)
    torch.cuda.synchronize()
    secs = (time.perf_counter() - t0) / steps
    return {"grid": [n, n, n], "ms_per_step": 1e3 * secs,
            "finite": bool(torch.isfinite(phi).all().item())}


def rd_workload(evx, torch, n: int = 256, steps: int = 100):
    """Single-species reaction-diffusion (logistic reaction, D = 1) on a 256^3 periodic spectral
    grid: ms per step (the stepper's four passes, the fused x pass evaluating the reaction)."""
    from paper_2507_21748_amd.inputs import quench_field
    shape = (n, n, n)
    plan = evx.Plan(shape, "periodic", "spectral")
    c = torch.from_numpy(quench_field(shape, 0.2, 0.1, seed=15)).cuda()
    prm = evx.RDParams(dt=0.5, D=1.0)
    plan.rd_step(c, 5, prm)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    plan.rd_step(c, steps, prm)
    torch.cuda.synchronize()
    secs = (time.perf_counter() - t0) / steps
    return {"grid": [n, n, n], "ms_per_step": 1e3 * secs,
            "finite": bool(torch.isfinite(c).all().item())}


def surrogate_workload(torch, w, reps: int = 5):
    """One coarse-stepper application (4 convolution layers, residual, mass projection) on the
    512^3 field: ms per application and the convolution flop rate (114,048 flop/voxel)."""
    from paper_2507_21748_amd.inputs import quench_field
    from paper_2507_21748_amd.surrogate import Net
    net = Net(seed=w.seed)
    c = torch.from_numpy(quench_field(w.shape, w.mean, w.amp, w.seed)).cuda()
    out = torch.empty_like(c)
    net.infer(c, out, conserve_mass=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.infer(c, out, conserve_mass=True)
    torch.cuda.synchronize()
    secs = (time.perf_counter() - t0) / reps
    flop = 114048.0 * w.voxels
    res = {"grid": list(w.shape[::-1]), "ms_per_application": 1e3 * secs,
           "conv_tflops": flop / secs / 1e12, "bf16_dense_peak_tflops": 2500.0,
           "finite": bool(torch.isfinite(out).all().item())}
    # one training step: batch 4 of 72^3 windows (64^3 interior, halo 4), forward, backward and
    # Adam; about 3x the forward flops per window voxel
    batch, edge, halo = 4, 72, 4
    x = torch.stack([torch.from_numpy(quench_field((edge,) * 3, 0.0, 0.5, 100 + i))
                     for i in range(batch)]).cuda()
    y = x.roll(1, dims=1).contiguous()
    net.train_step(x, y, halo, lr=1e-4)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        net.train_step(x, y, halo, lr=1e-4)
    torch.cuda.synchronize()
    tsecs = (time.perf_counter() - t0) / reps
    res["train_step_ms"] = 1e3 * tsecs
    res["train_window"] = [batch, edge, halo]
    res["train_conv_tflops"] = 3 * 114048.0 * batch * edge ** 3 / tsecs / 1e12
    del net, c, out, x, y
    torch.cuda.empty_cache()
    return res


def surrogate_experiment(torch):
    """The metric's third leg, surrogate against plain stepping at equal error: the network is
    trained on the GPU (600 Adam steps, batches of 4 windows of 72^3 from 256^3 solver
    trajectories), then a 512^3 quench is rolled to T = 500 by the network under each
    verification mode and by the plain solver at dt 0.5, 1, 2.5 and 5; errors are relative L2
    against the solver at dt 0.5."""
    from paper_2507_21748_amd import experiment
    net, info = experiment.train_network()
    res = experiment.surrogate_vs_plain(net)
    res["training"] = info
    del net
    torch.cuda.empty_cache()
    return res


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or "unknown"


def cpu_baseline():
    """FP64 oracle on this host: 2 timed steps (after 1 untimed) of a 512^3 periodic quench with
    the same physics and IC recipe as the benchmark workload."""
    import numpy as np
    from oracle import ch
    from paper_2507_21748_amd.inputs import quench_field
    # the host threads this process may use: OMP_NUM_THREADS where the host sets it (a shared
    # machine gives one GPU's processes a share of its cores), else every core the OS reports
    cores = int(os.environ.get("OMP_NUM_THREADS") or os.cpu_count() or 1)
    ch.WORKERS = cores
    p = ch.CHParams(dt=0.5)
    c = quench_field((512, 512, 512), 0.0, 0.05, 3).astype(np.float64)
    c = ch.ch_step(c, p, "periodic", "spectral")
    t0 = time.perf_counter()
    nsteps = 2
    for _ in range(nsteps):
        c = ch.ch_step(c, p, "periodic", "spectral")
    dt = time.perf_counter() - t0
    return {"value": 512 ** 3 * nsteps / dt, "unit": "voxel-steps/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(), "host_cpus": os.cpu_count(),
            "sample": "FP64 oracle (scipy.fft), 2 steps of a 512^3 periodic spectral quench "
                      "(mean 0, amp 0.05, dt 0.5) after 1 warm-up step"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--workload", default="ch1024_periodic")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extra", action="store_true")
    ap.add_argument("--copy-probe-gib", type=float, default=2.0,
                    help="size of the calibration copy run before the workload (0 = skip)")
    ap.add_argument("--summarize-profile", metavar="DIR",
                    help="summarize the rocprofv3 runs of PROFILE_COMMANDS found under DIR")
    ap.add_argument("--extra-only", choices=sorted(TRACE_COMMANDS),
                    help="run only this extra workload and print its JSON (for kernel traces)")
    ap.add_argument("--summarize-trace", metavar="DIR",
                    help="summarize the TRACE_COMMANDS run of --workload found under DIR")
    args = ap.parse_args()
    if args.summarize_profile:
        summarize_profile(args.summarize_profile, args.workload)
        return
    if args.summarize_trace:
        summarize_trace(args.summarize_trace, args.workload)
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU: the spectral stepper here runs on a single device "
              f"(--gpus {args.gpus} is not supported; multi-GPU sharding is design-only)",
              file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2507_21748_amd import evx
    from paper_2507_21748_amd.inputs import WORKLOADS
    evx.load()
    torch.cuda.set_device(0)
    if args.extra_only == "surrogate512":
        print(json.dumps({"surrogate512_application":
                          surrogate_workload(torch, WORKLOADS["surrogate512"])}))
        return
    if args.extra_only == "varmob256":
        print(json.dumps({"varmob256": varmob_workload(evx, torch, steps=20)}))
        return
    if args.extra_only == "inverse128":
        print(json.dumps({"inverse128_gradient":
                          adjoint_workload(evx, torch, WORKLOADS["inverse128"]),
                          "inverse128_gradient_stored":
                          adjoint_workload(evx, torch, WORKLOADS["inverse128"], every=0)}))
        return
    w = WORKLOADS[args.workload]
    probe = copy_probe(torch, args.copy_probe_gib) if args.copy_probe_gib > 0 else None
    res = run_workload(evx, torch, w, args.steps, args.warmup)
    passes = res["passes"]
    dom = max(passes, key=lambda k: passes[k]["avg_ms"] * passes[k]["launches"])
    d = passes[dom]
    roofline = {"bound": "hbm", "kernel": dom, "achieved": d["gbs"], "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": d["gbs"] / HBM_PEAK_GBS,
                "traffic": measured_traffic(w.name, dom),
                "bytes_per_launch": d["algorithmic_bytes"]}
    step_bytes = sum(pass_bytes(w.shape, w.bc))
    line = {
        "metric": "CH voxel-steps/s FP32 (semi-implicit Fourier-spectral step)",
        "value": res["voxel_steps_per_s"],
        "unit": "voxel-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": res["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic seeded quench field",
        "config": {"workload": w.name, "grid": list(w.shape[::-1]), "bc": w.bc,
                   "scheme": w.scheme, "dt": w.dt, "M": w.M, "kappa": w.kappa, "A": w.A,
                   "mean": w.mean, "amp": w.amp, "seed": w.seed, "parallelism": "single GPU"},
        "roofline": roofline,
        "step_effective_gbs": step_bytes * res["voxel_steps_per_s"] / w.voxels / 1e9,
        "passes": passes,
        "copy_probe": probe,
        "kernel_source_hash": kernel_source_hash(),
    }
    if not args.no_extra:
        extra = {}
        for name in ("ch256_periodic", "ch256_zeroflux", "ch400_zeroflux", "inverse128"):
            if name == args.workload:
                continue
            # step time without per-pass events (at these sizes the events add up to 25%),
            # then the per-pass times in a run of their own
            r = run_workload(evx, torch, WORKLOADS[name], 200, 10, timing=False)
            rp = run_workload(evx, torch, WORKLOADS[name], 50, 5, timing=True)
            wb = sum(pass_bytes(WORKLOADS[name].shape, WORKLOADS[name].bc))
            # the same loop with every kernel launched individually (the default replays
            # captured chunks of 8 steps on grids of at most 2^22 voxels)
            re = run_workload(evx, torch, WORKLOADS[name], 200, 10, timing=False, graph=0)
            extra[name] = {"voxel_steps_per_s": r["voxel_steps_per_s"],
                           "ms_per_step": r["ms_per_step"],
                           "ms_per_step_individual_launches": re["ms_per_step"],
                           "step_effective_gbs": wb * r["voxel_steps_per_s"]
                           / WORKLOADS[name].voxels / 1e9,
                           "passes": {k: v["avg_ms"] for k, v in rp["passes"].items()}}
        # the exponential (ETD1) stepper on the headline workload: same passes, the z pass's
        # update evaluates phi1(dt S) per bin
        r = run_workload(evx, torch, w, 50, 5, timing=False, integrator=evx.ETD1)
        extra[f"{w.name}_etd1"] = {"voxel_steps_per_s": r["voxel_steps_per_s"],
                                   "ms_per_step": r["ms_per_step"]}
        # the Allen-Cahn model on the same grid and passes (semi-implicit update)
        r = run_workload(evx, torch, w, 50, 5, timing=False, model=evx.ALLEN_CAHN)
        extra[f"{w.name}_allen_cahn"] = {"voxel_steps_per_s": r["voxel_steps_per_s"],
                                         "ms_per_step": r["ms_per_step"]}
        # Dirichlet boundary (DST-II) on the 256^3 stencil quench
        import dataclasses
        wd = dataclasses.replace(WORKLOADS["ch256_zeroflux"], name="ch256_dirichlet",
                                 bc="dirichlet")
        r = run_workload(evx, torch, wd, 200, 10, timing=False)
        extra["ch256_dirichlet"] = {"voxel_steps_per_s": r["voxel_steps_per_s"],
                                    "ms_per_step": r["ms_per_step"]}
        # vertex-centred zero flux (DCT-I as the periodic transform of the even extension) on
        # 257^3 points: 512-point y and z transforms, a 256-point complex x row
        wv = dataclasses.replace(WORKLOADS["ch256_zeroflux"], name="ch257_vertex",
                                 shape=(257, 257, 257), bc="zero_flux_vertex")
        r = run_workload(evx, torch, wv, 200, 10, timing=False)
        extra["ch257_vertex"] = {"voxel_steps_per_s": r["voxel_steps_per_s"],
                                 "ms_per_step": r["ms_per_step"],
                                 "workspace_bytes": r["workspace_bytes"]}
        extra["gray_scott256"] = gray_scott_workload(evx, torch)
        extra["varmob256"] = varmob_workload(evx, torch)
        extra["reaction_diffusion256"] = rd_workload(evx, torch)
        extra["inverse128_gradient"] = adjoint_workload(evx, torch, WORKLOADS["inverse128"])
        # the same with every state kept from the forward pass (1.7 GB): no recomputation
        extra["inverse128_gradient_stored"] = adjoint_workload(evx, torch, WORKLOADS["inverse128"],
                                                               every=0)
        extra["surrogate512_application"] = surrogate_workload(torch, WORKLOADS["surrogate512"])
        extra["surrogate_vs_plain"] = surrogate_experiment(torch)
        line["extra"] = extra
    if not args.no_cpu_baseline:
        cb = cpu_baseline()
        line["cpu_baseline"] = cb
        line["gpu_over_cpu"] = line["value"] / cb["value"]
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
