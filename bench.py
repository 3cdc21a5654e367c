#!/usr/bin/env python3
"""Benchmark: batched element-matrix integration on one MI355X.

Workload (the headline): 3D P1 linear elasticity on a 64^3-cell Kuhn-split unit
cube, 1,572,864 tetrahedra with 1% flattened to aspect ratio ~1e3, lognormal
per-element Lame coefficients, FP32 coordinates, inputs resident in HBM.

One step = one forward integration of the whole mesh in plain FP32
(gather -> J, J^-1, |J| -> geometric tensor -> G:K -> store).  ``value`` is
element matrices per second over the K timed steps.  The same protocol is
applied to further legs reported beside it: the split-precision MFMA forms,
the adjoint (dL/dA -> dL/dx, dL/dmu, dL/dlambda), and the 3D P1 Laplacian.
Kernel durations come from HIP events recorded on the launch stream around
every launch.  The CPU baseline is the FP64 oracle on the same workload; its
results also give the accuracy of every leg.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, vendor figure
METRIC = "element matrices/s + achieved GB/s, 3D P1 elasticity, plain FP32 vs MFMA form"


def kernel_source_digest() -> str:
    """Digest of the device sources; a stored traffic figure is only valid for it."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1103_0066_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def stored_traffic(kernel_tag: str):
    """HBM bytes per launch from profiles/traffic_<tag>.txt (rocprofv3 FETCH_SIZE +
    WRITE_SIZE, scaled by a plain copy of known size), or None if absent or
    taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"traffic_{kernel_tag}.txt")
    if not os.path.exists(path):
        return None
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_digest") != kernel_source_digest():
        return None
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense FP16/BF16 MFMA, vendor figure


def stored_mfma() -> dict:
    """MFMA flops per launch and busy fraction per precision from
    profiles/mfma_elastic_p1_3d_fwd.txt, if taken on the current sources."""
    path = os.path.join(ROOT, "profiles", "mfma_elastic_p1_3d_fwd.txt")
    if not os.path.exists(path):
        return {}
    vals = {}
    with open(path) as f:
        for line in f:
            if ":" in line and not line.startswith("#"):
                k, v = line.split(":", 1)
                vals[k.strip()] = v.strip()
    if vals.get("source_digest") != kernel_source_digest():
        return {}
    out = {}
    for prec in ("fp16x2", "bf16x2", "bf16x3"):
        try:
            out[prec] = {"flops": float(vals[f"{prec}_mfma_flops_per_launch"]),
                         "busy": float(vals[f"{prec}_mfma_busy_fraction"])}
        except (KeyError, ValueError):
            pass
    return out


def parse_args():
    p = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    p.add_argument("--gpus", type=int, default=1)
    p.add_argument("--steps", type=int, default=50)
    p.add_argument("--warmup", type=int, default=5)
    p.add_argument("--n", type=int, default=64, help="cells per side of the cube")
    p.add_argument("--legs", default="all",
                   help="'all', 'forward' (the FP32 and MFMA forward legs) or 'fp32' (headline only)")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--copy-ref", action="store_true",
                   help="also run a plain 512 MiB device copy (reference for PMC byte counters)")
    return p.parse_args()


def forward_bytes(E: int, n_vertices: int, n: int, dim: int, coeffs: bool, coord_bytes=4):
    """Compulsory HBM bytes of one forward pass: connectivity, coefficients and
    the output once per element, vertex coordinates once per vertex."""
    per_elem = 4 * (dim + 1) + (8 if coeffs else 0) + 4 * n * n
    return E * per_elem + n_vertices * dim * coord_bytes


def adjoint_bytes(E: int, n_vertices: int, n: int, dim: int, coeffs: bool):
    """dA, connectivity, coefficients and their gradients per element; vertex
    coordinates read once and the vertex gradient read and written once."""
    per_elem = 4 * n * n + 4 * (dim + 1) + (16 if coeffs else 0)
    return E * per_elem + n_vertices * dim * 4 * 3


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_leg(fn, steps: int, warmup: int, name: str = ""):
    import torch
    progress(f"leg {name}: {warmup} warmup + {steps} timed steps")
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for s, e in ev:
        s.record()
        fn()
        e.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    d = sorted(s.elapsed_time(e) for s, e in ev)
    return {
        "wall_ms_per_step": (t1 - t0) * 1e3 / steps,
        "kernel_ms_mean": sum(d) / len(d),
        "kernel_ms_median": d[len(d) // 2],
        "kernel_ms_p10": d[int(0.1 * (len(d) - 1))],
        "kernel_ms_p90": d[int(0.9 * (len(d) - 1))],
    }


def element_errors(A_gpu, A_orc):
    import numpy as np
    E = A_orc.shape[0]
    d = np.abs(A_gpu.reshape(E, -1).astype(np.float64) - A_orc.reshape(E, -1)).max(axis=1)
    return d / np.abs(A_orc.reshape(E, -1)).max(axis=1)


def batch_legs(fei, meshgen, dev, args):
    """The heterogeneous workload: 64 meshes, four forms, one graph launch per step."""
    import torch
    progress("generating the 64-mesh heterogeneous workload")
    wl = meshgen.batch_items()
    items, total_bytes, total_adj, E_tot = [], 0, 0, 0
    for k, w in enumerate(wl):
        m = w.mesh
        n = w.n_local
        it = {"form": w.form, "coords": torch.from_numpy(m.soa()).to(dev),
              "conn": torch.from_numpy(m.conn).to(dev)}
        el = w.mu is not None
        if el:
            it["mu"] = torch.from_numpy(w.mu).to(dev)
            it["lam"] = torch.from_numpy(w.lam).to(dev)
            it["dmu"] = torch.empty(m.n_elements, dtype=torch.float32, device=dev)
            it["dlam"] = torch.empty(m.n_elements, dtype=torch.float32, device=dev)
        it["dA"] = torch.from_numpy(meshgen.upstream(m.n_elements, n, 2000 + k)).to(dev)
        it["dcoords"] = torch.zeros((m.dim, m.n_vertices), dtype=torch.float32, device=dev)
        items.append(it)
        total_bytes += forward_bytes(m.n_elements, m.n_vertices, n, m.dim, el)
        total_adj += adjoint_bytes(m.n_elements, m.n_vertices, n, m.dim, el)
        E_tot += m.n_elements
    b = fei.Batch(items)
    out = {}
    for adj in (False, True):
        cfg = b.tune(adjoint=adj)
        fn = b.run_adjoint if adj else b.run
        r = time_leg(fn, args.steps, args.warmup, "batch_adjoint" if adj else "batch_forward")
        nb = total_adj if adj else total_bytes
        gbs = nb / (r["kernel_ms_mean"] * 1e-3) / 1e9
        out["batch_adjoint_fp32" if adj else "batch_forward_fp32"] = dict(
            r, gbs=gbs, frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=nb, elements=E_tot,
            meshes=len(items), elements_per_s=E_tot / (r["kernel_ms_mean"] * 1e-3),
            tuned_config=cfg,
            note="one hipGraphLaunch per step; time bracketed by events around the launch")
    b.close()
    return out


def main():
    args = parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU only: the library integrates on one device and has "
              "no cross-GPU step; run with --gpus 1.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    import meshgen
    import paper_1103_0066_amd as fei

    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    progress("generating the workload")
    w = meshgen.elast3d_adjoint(args.n)
    m = w.mesh
    E, Nv = m.n_elements, m.n_vertices
    coords = torch.from_numpy(m.soa()).to(dev)
    conn = torch.from_numpy(m.conn).to(dev)
    mu = torch.from_numpy(w.mu).to(dev)
    lam = torch.from_numpy(w.lam).to(dev)
    A = torch.empty((E, 12, 12), dtype=torch.float32, device=dev)
    fwd_bytes = forward_bytes(E, Nv, 12, 3, True)

    def fwd(prec):
        return lambda: fei.integrate(coords, conn, "elastic_p1", mu, lam, precision=prec, out=A)

    # ---- headline: plain FP32 forward -------------------------------------
    head = time_leg(fwd("fp32"), args.steps, args.warmup, "fp32")
    ms = head["wall_ms_per_step"]
    achieved = fwd_bytes / (head["kernel_ms_mean"] * 1e-3) / 1e9
    result = {
        "metric": METRIC,
        "value": E / (ms * 1e-3),
        "unit": "element matrices/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": w.name.replace("adjoint of ", ""), "elements": E,
                   "vertices": Nv, "precision": "fp32", "tau": 100.0,
                   "algorithmic_bytes_per_step": fwd_bytes},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": stored_traffic("elastic_p1_3d_fwd_fp32"),
                     "kernel": "fwd_fma_kernel<elastic_p1, 3, float, 12>",
                     "kernel_ms_mean": head["kernel_ms_mean"],
                     "algorithmic_bytes_per_launch": fwd_bytes},
    }
    legs = {"fp32": dict(head, gbs=achieved, elements_per_s=E / (head["kernel_ms_mean"] * 1e-3))}
    outputs = {}
    if args.legs in ("all", "forward"):
        mfma = stored_mfma()
        for prec in ("fp16x2", "bf16x2", "bf16x3"):
            r = time_leg(fwd(prec), args.steps, args.warmup, prec)
            gbs = fwd_bytes / (r["kernel_ms_mean"] * 1e-3) / 1e9
            legs[prec] = dict(r, gbs=gbs, frac=gbs / HBM_PEAK_GBS,
                              elements_per_s=E / (r["kernel_ms_mean"] * 1e-3),
                              speedup_vs_fp32=head["kernel_ms_mean"] / r["kernel_ms_mean"])
            if prec in mfma:
                fl = mfma[prec]["flops"]
                legs[prec]["mfma"] = {
                    "flops_per_launch": fl,
                    "achieved_tflops": fl / (r["kernel_ms_mean"] * 1e-3) / 1e12,
                    "peak_tflops": MFMA_PEAK_TFLOPS, "busy_fraction": mfma[prec]["busy"],
                    "source": "profiles/mfma_elastic_p1_3d_fwd.txt"}
    if args.legs == "all":
        # adjoint of the same workload
        dA = torch.from_numpy(w.dA).to(dev)
        dc = torch.zeros((3, Nv), dtype=torch.float32, device=dev)
        dmu = torch.empty(E, dtype=torch.float32, device=dev)
        dlam = torch.empty(E, dtype=torch.float32, device=dev)
        def adj():
            fei.integrate_adjoint(coords, conn, "elastic_p1", dA, mu, lam, dcoords=dc,
                                  dmu=dmu, dlam=dlam)
        r = time_leg(adj, args.steps, args.warmup, "adjoint_fp32")
        ab = adjoint_bytes(E, Nv, 12, 3, True)
        gbs = ab / (r["kernel_ms_mean"] * 1e-3) / 1e9
        legs["adjoint_fp32"] = dict(r, gbs=gbs, frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=ab,
                                    elements_per_s=E / (r["kernel_ms_mean"] * 1e-3))
        # the same adjoint through a one-mesh plan (tuned: atomic scatter or vertex gather)
        plan = fei.Batch([{"form": "elastic_p1", "coords": coords, "conn": conn, "mu": mu,
                           "lam": lam, "A": A, "dA": dA, "dcoords": dc, "dmu": dmu,
                           "dlam": dlam}])
        cfg = plan.tune(adjoint=True)
        r = time_leg(plan.run_adjoint, args.steps, args.warmup, "adjoint_plan_fp32")
        gbs = ab / (r["kernel_ms_mean"] * 1e-3) / 1e9
        legs["adjoint_plan_fp32"] = dict(
            r, gbs=gbs, frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=ab, tuned_config=cfg,
            elements_per_s=E / (r["kernel_ms_mean"] * 1e-3),
            note="one hipGraphLaunch per step (adjoint kernel, then the vertex gather when chosen)")
        plan.close()
        # 3D P1 Laplacian on the unflattened cube
        wl = meshgen.lap3d(args.n)
        cl = torch.from_numpy(wl.mesh.soa()).to(dev)
        kl = torch.from_numpy(wl.mesh.conn).to(dev)
        Al = torch.empty((wl.mesh.n_elements, 4, 4), dtype=torch.float32, device=dev)
        lb = forward_bytes(wl.mesh.n_elements, wl.mesh.n_vertices, 4, 3, False)
        for prec in ("fp32", "fp16x2"):
            r = time_leg(lambda: fei.integrate(cl, kl, "laplace_p1", precision=prec, out=Al),
                         args.steps, args.warmup, f"laplace3d_{prec}")
            gbs = lb / (r["kernel_ms_mean"] * 1e-3) / 1e9
            legs[f"laplace3d_{prec}"] = dict(
                r, gbs=gbs, frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=lb,
                elements_per_s=wl.mesh.n_elements / (r["kernel_ms_mean"] * 1e-3),
                note="129 MB working set fits the 256 MB MALL: GB/s here is not HBM-only")
        # 3D P1 Laplacian adjoint: single call (atomic scatter) and one-mesh plan
        dAl = torch.from_numpy(meshgen.upstream(wl.mesh.n_elements, 4, 1104)).to(dev)
        dcl = torch.zeros((3, wl.mesh.n_vertices), dtype=torch.float32, device=dev)
        lab = adjoint_bytes(wl.mesh.n_elements, wl.mesh.n_vertices, 4, 3, False)
        r = time_leg(lambda: fei.integrate_adjoint(cl, kl, "laplace_p1", dAl, dcoords=dcl),
                     args.steps, args.warmup, "laplace3d_adjoint_fp32")
        gbs = lab / (r["kernel_ms_mean"] * 1e-3) / 1e9
        legs["laplace3d_adjoint_fp32"] = dict(r, gbs=gbs, frac=gbs / HBM_PEAK_GBS,
                                              algorithmic_bytes=lab)
        plan = fei.Batch([{"form": "laplace_p1", "coords": cl, "conn": kl, "A": Al, "dA": dAl,
                           "dcoords": dcl}])
        cfg = plan.tune(adjoint=True)
        r = time_leg(plan.run_adjoint, args.steps, args.warmup, "laplace3d_adjoint_plan_fp32")
        gbs = lab / (r["kernel_ms_mean"] * 1e-3) / 1e9
        legs["laplace3d_adjoint_plan_fp32"] = dict(r, gbs=gbs, frac=gbs / HBM_PEAK_GBS,
                                                   algorithmic_bytes=lab, tuned_config=cfg)
        plan.close()
        del Al
        # 3D P2 Laplacian on the same unflattened cube (10 x 10 matrices)
        A2 = torch.empty((wl.mesh.n_elements, 10, 10), dtype=torch.float32, device=dev)
        pb = forward_bytes(wl.mesh.n_elements, wl.mesh.n_vertices, 10, 3, False)
        for prec in ("fp32", "fp16x2"):
            r = time_leg(lambda: fei.integrate(cl, kl, "laplace_p2", precision=prec, out=A2),
                         args.steps, args.warmup, f"laplace_p2_3d_{prec}")
            gbs = pb / (r["kernel_ms_mean"] * 1e-3) / 1e9
            legs[f"laplace_p2_3d_{prec}"] = dict(
                r, gbs=gbs, frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=pb,
                elements_per_s=wl.mesh.n_elements / (r["kernel_ms_mean"] * 1e-3))
        del A2
    if args.legs == "all":
        legs.update(batch_legs(fei, meshgen, dev, args))
    if args.copy_ref:
        n = 512 * 2**20 // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        r = time_leg(lambda: dst.copy_(src), args.steps, args.warmup, "copy_512MiB")
        legs["copy_512MiB_reference"] = dict(r, gbs=2 * n * 4 / (r["kernel_ms_mean"] * 1e-3) / 1e9)
        del src, dst
    result["legs"] = legs
    if not args.no_cpu_baseline and args.legs in ("all", "forward"):
        # outputs for the accuracy check, computed again and copied to the host
        # after every leg is timed (no large device-to-host copies between legs)
        for prec in ("fp32", "fp16x2", "bf16x2", "bf16x3"):
            fwd(prec)()
            outputs[prec] = A.cpu().numpy()

    # ---- CPU baseline: the FP64 oracle on the same workload ----------------
    if not args.no_cpu_baseline:
        import oracle
        cores = len(os.sched_getaffinity(0))
        threads = int(os.environ.get("OMP_NUM_THREADS", cores))
        progress(f"cpu baseline: FP64 oracle on {E} elements, {threads} threads")
        t0 = time.perf_counter()
        Ao = oracle.integrate("elastic_p1", m.coords, m.conn, w.mu, w.lam)
        t1 = time.perf_counter()
        # repeat whole passes until about 10 s of oracle time (bounded at 30 s)
        reps, total = 1, t1 - t0
        while total < 10.0 and total + (t1 - t0) < 30.0:
            ta = time.perf_counter()
            oracle.integrate("elastic_p1", m.coords, m.conn, w.mu, w.lam)
            total += time.perf_counter() - ta
            reps += 1
        result["cpu_baseline"] = {
            "value": reps * E / total, "unit": "element matrices/s",
            "cores": min(threads, cores), "kind": "oracle",
            "sample": f"{reps} pass(es) over the whole workload ({E} elements each), FP64 "
                      f"quadrature, OpenMP over elements, {total:.2f} s wall in total"}
        acc = {}
        for prec, Ag in outputs.items():
            if Ag is None:
                continue
            err = element_errors(Ag, Ao)
            acc[prec] = {"max": float(err.max()), "p99_9": float(np.quantile(err, 0.999)),
                         "median": float(np.median(err))}
        result["accuracy_vs_oracle"] = acc
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
