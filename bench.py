#!/usr/bin/env python3
"""Benchmark: batched element-matrix integration on one MI355X.

Workload (the headline): 3D P1 linear elasticity on a 64^3-cell Kuhn-split unit
cube, 1,572,864 tetrahedra with 1% flattened to aspect ratio ~1e3, lognormal
per-element Lame coefficients, FP32 coordinates, inputs resident in HBM.

One step = one forward integration of the whole mesh in plain FP32
(gather -> J, J^-1, |J| -> geometric tensor -> G:K -> store).  ``value`` is
element matrices per second over the K timed steps.  The same protocol is
applied to further legs reported beside it: the split-precision MFMA forms,
the adjoint (dL/dA -> dL/dx, dL/dmu, dL/dlambda) as a single call, in its
deterministic form and through a one-mesh plan, the 3D P1 and P2 Laplacians,
the 2D P1 Laplacian with FP64 coordinates (a latency-bound size), and the
64-mesh heterogeneous batch.

Timing protocol: consecutive timed launches of a leg cycle through several
independent copies of its inputs and outputs (together well above twice the
256 MB last-level cache), so no launch finds the previous one's data in the
cache; every launch is bracketed by HIP events on the launch stream.  GB/s are
algorithmic bytes (compulsory HBM traffic) over the mean event time, reported
against the 8 TB/s vendor figure and against a measured 512 MiB device copy.
The CPU baseline is the FP64 oracle on the same workload (all host cores, and
one core on a bounded sample); its results also give every leg's accuracy.
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

HBM_PEAK_GBS = 8000.0      # MI355X HBM3E, vendor figure
MFMA_PEAK_TFLOPS = 2500.0  # MI355X dense FP16/BF16 MFMA, vendor figure
MALL_BYTES = 256 * 2**20   # last-level (Infinity) cache
METRIC = "element matrices/s + achieved GB/s, 3D P1 elasticity, plain FP32 vs MFMA form"


def kernel_source_digest() -> str:
    """Digest of the device sources; a stored counter figure is only valid for it."""
    import hashlib
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_1103_0066_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        if name.endswith((".h", ".hip", ".cpp")):
            with open(os.path.join(csrc, name), "rb") as f:
                h.update(name.encode() + b"\0" + f.read())
    return h.hexdigest()[:16]


def _profile_values(name: str) -> dict:
    path = os.path.join(ROOT, "profiles", name)
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
    return vals


def stored_traffic(leg: str):
    """HBM bytes per launch of a leg from profiles/traffic_<leg>.txt (rocprofv3
    FETCH_SIZE + WRITE_SIZE, scaled by a plain copy of known size), or None if
    absent or taken on other kernel sources."""
    vals = _profile_values(f"traffic_{leg}.txt")
    try:
        return float(vals["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


def stored_mfma() -> dict:
    """MFMA flops per launch and busy fraction per precision from
    profiles/mfma_elastic_p1_3d_fwd.txt, if taken on the current sources."""
    vals = _profile_values("mfma_elastic_p1_3d_fwd.txt")
    out = {}
    for prec in ("fp16x2", "bf16x2", "bf16x3"):
        for key in (prec, f"adjoint_{prec}"):
            try:
                out[key] = {"flops": float(vals[f"{key}_mfma_flops_per_launch"]),
                            "busy": float(vals[f"{key}_mfma_busy_fraction"])}
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
                   help="'all', 'forward' (the FP32 and MFMA forward legs), 'fp32' (headline "
                        "only), or a comma-separated list of leg names")
    p.add_argument("--no-cpu-baseline", action="store_true")
    p.add_argument("--no-accuracy", action="store_true",
                   help="skip the oracle comparisons of the legs' outputs")
    p.add_argument("--sets", type=int, default=4,
                   help="independent input/output copies cycled through by the timed launches")
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


def paper_flops(dim: int, n: int) -> int:
    """The paper's flop convention per element: the d x d contraction of every
    one of the n^2 entries, 2 d^2 n^2 (Sec. 4.3's per-entry block product)."""
    return 2 * dim * dim * n * n


def progress(msg: str):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def time_leg(fns, steps: int, warmup: int, name: str = ""):
    """Times ``steps`` launches; launch k calls fns[k % len(fns)] (each a
    different copy of the leg's buffers)."""
    import torch
    if callable(fns):
        fns = [fns]
    progress(f"leg {name}: {warmup} warmup + {steps} timed launches over {len(fns)} buffer set(s)")
    for k in range(warmup):
        fns[k % len(fns)]()
    torch.cuda.synchronize()
    # the timed steps: back to back, bracketed by synchronizations (wall clock)
    # and by one pair of events on the launch stream
    r0, r1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    r0.record()
    for k in range(steps):
        fns[k % len(fns)]()
    r1.record()
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    # per-launch durations: the same launches again, each between two events
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(steps)]
    for k, (s, e) in enumerate(ev):
        s.record()
        fns[k % len(fns)]()
        e.record()
    torch.cuda.synchronize()
    d = sorted(s.elapsed_time(e) for s, e in ev)
    return {
        "wall_ms_per_step": (t1 - t0) * 1e3 / steps,
        # mean duration of a launch over the timed region (HIP events on the
        # launch stream around the K back-to-back steps): the rates use this
        "ms_per_launch": r0.elapsed_time(r1) / steps,
        "kernel_ms_mean": sum(d) / len(d),
        "kernel_ms_median": d[len(d) // 2],
        "kernel_ms_p10": d[int(0.1 * (len(d) - 1))],
        "kernel_ms_p90": d[int(0.9 * (len(d) - 1))],
        "buffer_sets": len(fns),
    }


def rates(r: dict, nbytes: int, E: int, flops_per_elem: int = 0, copy_gbs=None, traffic=None):
    """GB/s, roofline fractions, elements/s and paper-convention GF/s of a leg."""
    t = r["ms_per_launch"] * 1e-3
    gbs = nbytes / t / 1e9
    out = dict(r, gbs=gbs, frac=gbs / HBM_PEAK_GBS, algorithmic_bytes=nbytes,
               elements=E, elements_per_s=E / t)
    if flops_per_elem:
        out["gflops_paper_convention"] = flops_per_elem * E / t / 1e9
    if copy_gbs:
        out["frac_of_measured_copy"] = gbs / copy_gbs
    if traffic is not None:
        out["traffic_bytes_per_launch"] = traffic
        out["traffic_over_algorithmic"] = traffic / nbytes
    return out


def element_errors(A_gpu, A_orc):
    import numpy as np
    E = A_orc.shape[0]
    d = np.abs(A_gpu.reshape(E, -1).astype(np.float64) - A_orc.reshape(E, -1)).max(axis=1)
    return d / np.abs(A_orc.reshape(E, -1)).max(axis=1)


def error_summary(err):
    import numpy as np
    return {"max": float(err.max()), "p99_9": float(np.quantile(err, 0.999)),
            "median": float(np.median(err)), "count": int(err.size)}


def adjoint_accuracy(oracle, mesh, form, g, dA, mu, lam, dmu=None, dlam=None, nverts=200,
                     nelems=2000, seed=5):
    """Vertex gradients g [N_v, dim] at sampled vertices against the oracle over all
    their incident elements (error relative to the sum of the incident elements'
    gradient norms); coefficient gradients at sampled elements, relative to
    sum |dA| |dA/dmu| (resp. lambda)."""
    import numpy as np
    rng = np.random.Generator(np.random.PCG64(seed))
    verts = rng.choice(mesh.n_vertices, min(nverts, mesh.n_vertices), replace=False)
    inc = np.nonzero(np.isin(mesh.conn, verts).any(axis=1))[0]
    sel = (lambda a: None if a is None else a[inc])
    gv, _, _, _ = oracle.gradient(form, mesh.coords, mesh.conn[inc], dA[inc], sel(mu), sel(lam))
    go = oracle.vertex_gradient(gv, mesh.conn[inc], mesh.n_vertices)[verts]
    mag = np.abs(gv).reshape(len(inc), -1).max(axis=1)      # norm of each element's gradient
    sc = np.zeros(mesh.n_vertices)
    np.add.at(sc, mesh.conn[inc].ravel(), np.repeat(mag, mesh.conn.shape[1]))
    sc = sc[verts]
    ok = sc > 0
    verr = np.abs(g[verts] - go).max(axis=1)[ok] / sc[ok]
    out = {"vertex": error_summary(verr), "sampled_vertices": int(ok.sum())}
    if dmu is not None:
        idx = rng.choice(mesh.n_elements, min(nelems, mesh.n_elements), replace=False)
        _, gm, gl, _ = oracle.gradient(form, mesh.coords, mesh.conn[idx], dA[idx], mu[idx],
                                       lam[idx])
        d2 = np.abs(dA[idx]).reshape(len(idx), -1)
        one, zero = np.ones(len(idx)), np.zeros(len(idx))
        Am = np.abs(oracle.integrate(form, mesh.coords, mesh.conn[idx], one, zero)).reshape(len(idx), -1)
        Al = np.abs(oracle.integrate(form, mesh.coords, mesh.conn[idx], zero, one)).reshape(len(idx), -1)
        cerr = np.maximum(np.abs(dmu[idx] - gm) / (d2 * Am).sum(axis=1),
                          np.abs(dlam[idx] - gl) / (d2 * Al).sum(axis=1))
        out["coefficients"] = error_summary(cerr)
    return out


def replicate(torch, dev, arrays, sets):
    """``sets`` device copies of a tuple of host arrays (None stays None)."""
    out = []
    for _ in range(sets):
        out.append(tuple(None if a is None else torch.from_numpy(a).to(dev) for a in arrays))
    return out


def want(args, name, group):
    if args.legs == "all":
        return True
    if args.legs == "forward":
        return group == "forward"
    if args.legs == "fp32":
        return name == "fp32"
    return name in args.legs.split(",")


def batch_legs(fei, meshgen, oracle, dev, args, legs, copy_gbs, acc):
    """The heterogeneous workload: 64 meshes, four forms, one graph launch per step.
    Its outputs (1.7 GB per forward) exceed the last-level cache many times over,
    so one buffer set suffices."""
    import numpy as np
    import torch
    progress("generating the 64-mesh heterogeneous workload")
    wl = meshgen.batch_items()
    items, total_bytes, total_adj, E_tot, fl = [], 0, 0, 0, 0
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
        it["dA_host"] = meshgen.upstream(m.n_elements, n, 2000 + k)
        it["dA"] = torch.from_numpy(it["dA_host"]).to(dev)
        it["dcoords"] = torch.zeros((m.dim, m.n_vertices), dtype=torch.float32, device=dev)
        items.append(it)
        total_bytes += forward_bytes(m.n_elements, m.n_vertices, n, m.dim, el)
        total_adj += adjoint_bytes(m.n_elements, m.n_vertices, n, m.dim, el)
        E_tot += m.n_elements
        fl += paper_flops(m.dim, n) * m.n_elements
    b = fei.Batch(items)
    for adj in (False, True):
        name = "batch_adjoint_fp32" if adj else "batch_forward_fp32"
        cfg = b.tune(adjoint=adj)
        fn = b.run_adjoint if adj else b.run
        r = time_leg(fn, args.steps, args.warmup, name)
        nb = total_adj if adj else total_bytes
        legs[name] = rates(r, nb, E_tot, 0, copy_gbs, stored_traffic(name))
        legs[name].update(meshes=len(items), tuned_config=cfg,
                          gflops_paper_convention=fl / (r["ms_per_launch"] * 1e-3) / 1e9,
                          note="one hipGraphLaunch per step; events around the launch")
    if not args.no_accuracy:
        # forward: sampled elements of every mesh; adjoint: one clean run, sampled
        b.run()
        for it in items:
            it["dcoords"].zero_()
        b.run_adjoint()
        torch.cuda.synchronize()
        rng = np.random.Generator(np.random.PCG64(3))
        fe, ve, ce = [], [], []
        for w, it in zip(wl, items):
            m = w.mesh
            idx = np.union1d(rng.choice(m.n_elements, min(100, m.n_elements), replace=False),
                             [m.n_elements - 1])
            A = it["A"][torch.from_numpy(idx).to(dev)].cpu().numpy()
            Ao = oracle.integrate(w.form, m.coords, m.conn[idx],
                                  None if w.mu is None else w.mu[idx],
                                  None if w.lam is None else w.lam[idx])
            fe.append(element_errors(A, Ao))
            g = it["dcoords"].cpu().numpy().T.astype(np.float64)
            a = adjoint_accuracy(oracle, m, w.form, g, it["dA_host"], w.mu, w.lam,
                                 None if w.mu is None else it["dmu"].cpu().numpy(),
                                 None if w.lam is None else it["dlam"].cpu().numpy(),
                                 nverts=20, nelems=50, seed=7)
            ve.append(a["vertex"]["max"])
            if "coefficients" in a:
                ce.append(a["coefficients"]["max"])
        acc["batch_forward_fp32"] = error_summary(np.concatenate(fe))
        acc["batch_adjoint_fp32"] = {"vertex_max": float(max(ve)), "coefficients_max":
                                     float(max(ce)) if ce else None,
                                     "sample": "20 vertices and 50 elements per mesh"}
    b.close()


def assembly_legs(fei, meshgen, dev, args, legs, copy_gbs, acc):
    """Fused global assembly (the global sparse matrix, element matrices never
    stored) of 3D P1 elasticity and the 3D P1 Laplacian on the 64^3 cube, and
    the Laplacian with a P1 coefficient w (element matrices, eqs. 20-23)."""
    import numpy as np
    import torch
    for name, make in (("assembly_elastic_p1_3d", lambda: meshgen.elast3d(args.n)),
                       ("assembly_laplace_p1_3d", lambda: meshgen.lap3d(args.n))):
        if not want(args, name, "assembly"):
            continue
        progress(f"{name}: building the plan")
        w = make()
        m = w.mesh
        el = w.mu is not None
        coords = torch.from_numpy(m.soa()).to(dev)
        conn = torch.from_numpy(m.conn).to(dev)
        mu = torch.from_numpy(w.mu).to(dev) if el else None
        lam = torch.from_numpy(w.lam).to(dev) if el else None
        asm = fei.Assembly(coords, conn, w.form)
        nc = asm.block
        # values (written once), conn, mu/lam, coordinates, pattern (rowptr, colidx),
        # incidence (ptr, inc) once each
        nbytes = (asm.nnz * nc * nc * 4 + m.conn.nbytes + (8 * m.n_elements if el else 0)
                  + m.n_vertices * 3 * 4 + 4 * (asm.n_rows + 1) + 4 * asm.nnz
                  + 4 * (m.n_vertices + 1) + 4 * m.conn.size)
        # enough value arrays that the cycle exceeds twice the cache
        S = max(2, -(-2 * MALL_BYTES // (asm.nnz * nc * nc * 4)) + 1)
        outs = [torch.empty((asm.nnz, nc, nc), dtype=torch.float32, device=dev) for _ in range(S)]
        fns = [(lambda k=k: asm.assemble(mu, lam, out=outs[k])) for k in range(S)]
        r = time_leg(fns, args.steps, args.warmup, name)
        legs[name] = rates(r, nbytes, m.n_elements, 0, copy_gbs, stored_traffic(name))
        legs[name].update(nnz_blocks=asm.nnz, block=nc, output_sets=S,
                          note="element matrices/s counts the elements integrated into the "
                               "global matrix per launch")
        if not args.no_accuracy:
            import oracle
            import scipy.sparse as sp
            fns[0]()
            rowptr, colidx = asm.pattern()
            vals = outs[0].cpu().numpy()
            K = sp.bsr_matrix((vals, colidx.cpu().numpy(), rowptr.cpu().numpy()),
                              shape=(nc * asm.n_rows,) * 2).tocsr()
            rng = np.random.Generator(np.random.PCG64(11))
            verts = rng.choice(m.n_vertices, 200, replace=False)
            inc = np.nonzero(np.isin(m.conn, verts).any(axis=1))[0]
            sel = (lambda a: None if a is None else a[inc])
            Ko = oracle.assemble(w.form, m.coords, m.conn[inc], sel(w.mu), sel(w.lam))
            Ae = oracle.integrate(w.form, m.coords, m.conn[inc], sel(w.mu), sel(w.lam))
            nrm = np.abs(Ae).reshape(len(inc), -1).max(axis=1)
            dofs = (nc * m.conn[inc].astype(np.int64)[:, :, None] + np.arange(nc)).reshape(len(inc), -1)
            nl = dofs.shape[1]
            Sc = sp.coo_matrix((np.repeat(nrm, nl * nl), (np.repeat(dofs, nl, axis=1).ravel(),
                                                         np.tile(dofs, (1, nl)).ravel())),
                               shape=Ko.shape).tocsr()
            rows = (nc * verts[:, None] + np.arange(nc)).ravel()
            Kr, Kor, Sr = K[rows], Ko[rows], Sc[rows]
            for X in (Kr, Kor, Sr):
                X.sort_indices()
            err = np.abs(Kr.data - Kor.data) / Sr.data
            acc[name] = dict(error_summary(err), sample="200 block rows; error relative to the "
                             "sum of the contributing element matrices' norms")
        asm.close()
        del outs
        torch.cuda.empty_cache()
    name = "coefficient_laplace_p1_3d"
    if want(args, name, "assembly"):
        wl = meshgen.lap3d(args.n)
        ml = wl.mesh
        El, Nl = ml.n_elements, ml.n_vertices
        wv = np.exp(0.5 * np.random.Generator(np.random.PCG64(12)).standard_normal(Nl)).astype(np.float32)
        nbytes = forward_bytes(El, Nl, 4, 3, False) + 4 * Nl
        S = max(2, -(-2 * MALL_BYTES // nbytes) + 1)
        sets = replicate(torch, dev, (ml.soa(), ml.conn, wv), S)
        outs = [torch.empty((El, 4, 4), dtype=torch.float32, device=dev) for _ in range(S)]
        fns = [(lambda k=k: fei.integrate_coefficient(sets[k][0], sets[k][1], "laplace_p1",
                                                      sets[k][2], out=outs[k])) for k in range(S)]
        r = time_leg(fns, args.steps, args.warmup, name)
        legs[name] = rates(r, nbytes, El, paper_flops(3, 4) * 4, copy_gbs, stored_traffic(name))
        legs[name]["note"] = ("A_ij = int w grad phi_i . grad phi_j, w in P1 (arity-3 K); "
                              "paper-convention flops 2 d^2 n^2 (d + 1) per element")
        if not args.no_accuracy:
            import oracle
            idx = np.sort(np.random.Generator(np.random.PCG64(13)).choice(El, 50000, replace=False))
            fns[0]()
            Ag = outs[0][torch.from_numpy(idx).to(dev)].cpu().numpy()
            Ao = oracle.integrate_coefficient("laplace_p1", ml.coords, ml.conn[idx], wv)
            acc[name] = dict(error_summary(element_errors(Ag, Ao)), sample="50,000 elements")
        del sets, outs
        torch.cuda.empty_cache()


def iso_leg(fei, meshgen, dev, args, legs, copy_gbs, acc):
    """The isoparametric P2 Laplacian (Sec. 3.1, eqs. 16-19) on the 64^3 Kuhn
    cube with curved (quadratic) edges: 10 nodes and a 10 x 10 matrix per tet."""
    import numpy as np
    import torch
    name = "iso_p2_3d"
    progress(f"{name}: generating the curved mesh")
    w = meshgen.iso3d(args.n)
    m = w.mesh
    E = m.n_elements
    nbytes = E * (m.conn.shape[1] * 4 + 400) + m.n_vertices * 12
    S = max(2, -(-2 * MALL_BYTES // nbytes) + 1)
    sets = replicate(torch, dev, (m.soa(), m.conn), S)
    outs = [torch.empty((E, 10, 10), dtype=torch.float32, device=dev) for _ in range(S)]
    fns = [(lambda k=k: fei.integrate_iso(sets[k][0], sets[k][1], out=outs[k])) for k in range(S)]
    r = time_leg(fns, args.steps, args.warmup, name)
    # the dense contraction of eq. 19: (d+1)^2 d^2 terms for each of the n^2 entries
    legs[name] = rates(r, nbytes, E, 2 * 16 * 9 * 100, copy_gbs, stored_traffic(name))
    legs[name].update(nodes=m.n_vertices, note=(
        "paper-convention flops: 2 (d+1)^2 d^2 n^2 per element (eq. 19's contraction)"))
    if not args.no_accuracy:
        import oracle
        idx = np.sort(np.random.Generator(np.random.PCG64(15)).choice(E, 50000, replace=False))
        fns[0]()
        Ag = outs[0][torch.from_numpy(idx).to(dev)].cpu().numpy()
        Ao = oracle.integrate_iso(m.coords, m.conn[idx])
        acc[name] = dict(error_summary(element_errors(Ag, Ao)), sample="50,000 elements")
    del sets, outs
    torch.cuda.empty_cache()


def form_leg(fei, meshgen, dev, args, legs, copy_gbs, acc, S):
    """The headline elasticity written in the form language and integrated by
    the front end's generic kernel (runtime Khat and recipe), beside the
    specialized kernel of the fp32 leg."""
    import numpy as np
    import torch
    from paper_1103_0066_amd import forms as F
    name = "form_elastic_p1_3d"
    el = F.Element(3, 1, vector=True)
    u, v = F.TrialFunction(el), F.TestFunction(el)
    mu, lam = F.Coefficient("mu"), F.Coefficient("lam")
    form = F.compile_form(2 * mu * F.inner(F.eps(u), F.eps(v)) + lam * F.div(u) * F.div(v))
    generic = F.compile_form(2 * mu * F.inner(F.eps(u), F.eps(v)) + lam * F.div(u) * F.div(v))
    progress(f"{name}: generating and compiling the form's kernel")
    form.compile()
    w = meshgen.elast3d(args.n)
    m = w.mesh
    E = m.n_elements
    sets = replicate(torch, dev, (m.soa(), m.conn, w.mu, w.lam), S)
    outs = [torch.empty((E, 12, 12), dtype=torch.float32, device=dev) for _ in range(S)]
    fns = [(lambda k=k: form.integrate(sets[k][0], sets[k][1],
                                       {"mu": sets[k][2], "lam": sets[k][3]}, out=outs[k]))
           for k in range(S)]
    r = time_leg(fns, args.steps, args.warmup, name)
    nb = forward_bytes(E, m.n_vertices, 12, 3, True)
    legs[name] = rates(r, nb, E, paper_flops(3, 12), copy_gbs, stored_traffic(name))
    legs[name]["note"] = ("2 mu inner(eps(u), eps(v)) + lam div(u) div(v) through the form front "
                          "end, with the kernel it generates and compiles for the form (W and Khat "
                          "as constants; fei_form_compile)")
    # the same form through the generic kernel (tables read at run time)
    gfns = [(lambda k=k: generic.integrate(sets[k][0], sets[k][1],
                                           {"mu": sets[k][2], "lam": sets[k][3]}, out=outs[k]))
            for k in range(S)]
    rg = time_leg(gfns, args.steps, args.warmup, name + "_generic")
    legs[name + "_generic"] = rates(rg, nb, E, paper_flops(3, 12), copy_gbs,
                                    stored_traffic(name + "_generic"))
    legs[name + "_generic"]["note"] = "the same form through the generic kernel (W, Khat at run time)"
    generic.close()
    if not args.no_accuracy:
        import oracle
        idx = np.sort(np.random.Generator(np.random.PCG64(14)).choice(E, 50000, replace=False))
        fns[0]()
        Ag = outs[0][torch.from_numpy(idx).to(dev)].cpu().numpy()
        Ao = oracle.integrate("elastic_p1", m.coords, m.conn[idx], w.mu[idx], w.lam[idx])
        acc[name] = dict(error_summary(element_errors(Ag, Ao)), sample="50,000 elements")
    form.close()
    del sets, outs
    torch.cuda.empty_cache()


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
    S = max(1, args.sets)
    legs, acc = {}, {}

    # ---- reference: a plain device copy ------------------------------------
    copy_gbs = None
    if args.legs in ("all", "forward") or want(args, "copy_512MiB", "ref"):
        n = 512 * 2**20 // 4
        src = torch.ones(n, dtype=torch.float32, device=dev)
        dst = torch.empty_like(src)
        r = time_leg(lambda: dst.copy_(src), args.steps, args.warmup, "copy_512MiB")
        copy_gbs = 2 * n * 4 / (r["ms_per_launch"] * 1e-3) / 1e9
        legs["copy_512MiB_reference"] = dict(r, gbs=copy_gbs, frac=copy_gbs / HBM_PEAK_GBS,
                                             traffic_bytes_per_launch=2 * n * 4)
        del src, dst

    progress("generating the workload")
    w = meshgen.elast3d_adjoint(args.n)
    m = w.mesh
    E, Nv = m.n_elements, m.n_vertices
    fwd_bytes = forward_bytes(E, Nv, 12, 3, True)
    sets = replicate(torch, dev, (m.soa(), m.conn, w.mu, w.lam), S)
    outs = [torch.empty((E, 12, 12), dtype=torch.float32, device=dev) for _ in range(S)]
    pf = paper_flops(3, 12)

    def fwd(prec, k):
        c, cn, mu, lam = sets[k]
        return lambda: fei.integrate(c, cn, "elastic_p1", mu, lam, precision=prec, out=outs[k])

    # ---- headline: plain FP32 forward, launch shape from the tuner ---------
    # (fei_tune_forward times the elements-per-workgroup and staging
    # candidates on this mesh and records the fastest; the timed calls below
    # take it from the tune table)
    c0, cn0, mu0, lam0 = sets[0]
    tuned = fei.tune_forward(c0, cn0, "elastic_p1", mu0, lam0, out=outs[0])
    progress(f"tuned launch shape of the headline forward: {tuned}")
    blk = tuned["block_elements"] or 256            # 0 in the table: the built-in default
    rows = tuned["store_rows"] or 12
    head = time_leg([fwd("fp32", k) for k in range(S)], args.steps, args.warmup, "fp32")
    ms = head["wall_ms_per_step"]
    achieved = fwd_bytes / (head["ms_per_launch"] * 1e-3) / 1e9
    head_traffic = stored_traffic("elastic_p1_3d_fwd_fp32")
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
                   "algorithmic_bytes_per_step": fwd_bytes, "buffer_sets": S,
                   "tuned_launch": {"block_elements": blk, "store_rows": rows}},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": achieved / HBM_PEAK_GBS,
                     "traffic": head_traffic,
                     "kernel": f"fwd_fma_kernel<elastic_p1, 3, float, {rows}, {blk // 64}>",
                     "ms_per_launch": head["ms_per_launch"],
                     "kernel_ms_mean_event_pairs": head["kernel_ms_mean"],
                     "algorithmic_bytes_per_launch": fwd_bytes},
    }
    legs["fp32"] = rates(head, fwd_bytes, E, pf, copy_gbs, head_traffic)
    if copy_gbs:
        result["roofline"]["frac_of_measured_copy"] = achieved / copy_gbs
        result["roofline"]["measured_copy_gbs"] = copy_gbs

    mfma = stored_mfma()
    for prec in ("fp16x2", "bf16x2", "bf16x3"):
        if not want(args, prec, "forward"):
            continue
        r = time_leg([fwd(prec, k) for k in range(S)], args.steps, args.warmup, prec)
        legs[prec] = rates(r, fwd_bytes, E, pf, copy_gbs,
                           stored_traffic(f"elastic_p1_3d_fwd_{prec}"))
        legs[prec]["speedup_vs_fp32"] = head["ms_per_launch"] / r["ms_per_launch"]
        if prec in mfma:
            fl = mfma[prec]["flops"]
            legs[prec]["mfma"] = {
                "flops_per_launch": fl,
                "achieved_tflops": fl / (r["ms_per_launch"] * 1e-3) / 1e12,
                "peak_tflops": MFMA_PEAK_TFLOPS, "busy_fraction": mfma[prec]["busy"],
                "source": "profiles/mfma_elastic_p1_3d_fwd.txt"}

    # ---- adjoint of the same workload ------------------------------------------
    ab = adjoint_bytes(E, Nv, 12, 3, True)
    if any(want(args, k, "adjoint") for k in ("adjoint_fp32", "adjoint_det_fp32",
                                              "adjoint_plan_fp32", "adjoint_fp16x2",
                                              "adjoint_bf16x2", "adjoint_bf16x3")):
        A_plan = outs[0]            # the plans' forward output (their forward is not run)
        del outs
        torch.cuda.empty_cache()
        dAs = [torch.from_numpy(w.dA).to(dev) for _ in range(S)]
        dcs = [torch.zeros((3, Nv), dtype=torch.float32, device=dev) for _ in range(S)]
        dmus = [torch.empty(E, dtype=torch.float32, device=dev) for _ in range(S)]
        dlams = [torch.empty(E, dtype=torch.float32, device=dev) for _ in range(S)]

        def adj(k, det=False, prec="fp32"):
            c, cn, mu, lam = sets[k]
            return lambda: fei.integrate_adjoint(c, cn, "elastic_p1", dAs[k], mu, lam,
                                                 dcoords=dcs[k], dmu=dmus[k], dlam=dlams[k],
                                                 deterministic=det, precision=prec)

        def adj_acc(name, run):
            if args.no_accuracy:
                return
            import oracle
            dcs[0].zero_()
            run()
            torch.cuda.synchronize()
            acc[name] = adjoint_accuracy(oracle, m, "elastic_p1", dcs[0].cpu().numpy().T.astype(np.float64),
                                         w.dA, w.mu, w.lam, dmus[0].cpu().numpy(),
                                         dlams[0].cpu().numpy())

        if want(args, "adjoint_fp32", "adjoint"):
            r = time_leg([adj(k) for k in range(S)], args.steps, args.warmup, "adjoint_fp32")
            legs["adjoint_fp32"] = rates(r, ab, E, 0, copy_gbs,
                                         stored_traffic("elastic_p1_3d_adjoint_fp32"))
            adj_acc("adjoint_fp32", adj(0))
        for prec in ("fp16x2", "bf16x2", "bf16x3"):
            name = f"adjoint_{prec}"
            if not want(args, name, "adjoint"):
                continue
            r = time_leg([adj(k, prec=prec) for k in range(S)], args.steps, args.warmup, name)
            legs[name] = rates(r, ab, E, 0, copy_gbs,
                               stored_traffic(f"elastic_p1_3d_adjoint_{prec}"))
            legs[name]["note"] = ("the fold of dA with K on the matrix cores, dA split into "
                                  "16-bit terms; whole-matrix staging; atomic vertex scatter")
            if "adjoint_fp32" in legs:
                legs[name]["speedup_vs_fp32"] = (legs["adjoint_fp32"]["ms_per_launch"]
                                                 / legs[name]["ms_per_launch"])
            if name in mfma:
                fl = mfma[name]["flops"]
                legs[name]["mfma"] = {
                    "flops_per_launch": fl,
                    "achieved_tflops": fl / (r["ms_per_launch"] * 1e-3) / 1e12,
                    "peak_tflops": MFMA_PEAK_TFLOPS, "busy_fraction": mfma[name]["busy"],
                    "source": "profiles/mfma_elastic_p1_3d_fwd.txt"}
            adj_acc(name, adj(0, prec=prec))
        if want(args, "adjoint_det_fp32", "adjoint"):
            r = time_leg([adj(k, True) for k in range(S)], args.steps, args.warmup,
                         "adjoint_det_fp32")
            legs["adjoint_det_fp32"] = rates(r, ab, E, 0, copy_gbs)
            legs["adjoint_det_fp32"]["note"] = (
                "deterministic single call: incidence build + J-bar adjoint + vertex gather "
                "per call; algorithmic bytes as the adjoint's")
            adj_acc("adjoint_det_fp32", adj(0, True))
        if want(args, "adjoint_plan_fp32", "adjoint"):
            plans = []
            for k in range(S):
                c, cn, mu, lam = sets[k]
                plans.append(fei.Batch([{"form": "elastic_p1", "coords": c, "conn": cn, "mu": mu,
                                         "lam": lam, "A": A_plan, "dA": dAs[k],
                                         "dcoords": dcs[k], "dmu": dmus[k], "dlam": dlams[k]}]))
            cfg = plans[0].tune(adjoint=True)
            for p in plans[1:]:
                p.set_config(cfg, adjoint=True)
            r = time_leg([p.run_adjoint for p in plans], args.steps, args.warmup,
                         "adjoint_plan_fp32")
            legs["adjoint_plan_fp32"] = rates(r, ab, E, 0, copy_gbs,
                                              stored_traffic("elastic_p1_3d_adjoint_plan_fp32"))
            legs["adjoint_plan_fp32"].update(
                tuned_config=cfg,
                note="one hipGraphLaunch per step (adjoint kernel, then the vertex gather "
                     "when chosen)")
            adj_acc("adjoint_plan_fp32", plans[0].run_adjoint)
            for p in plans:
                p.close()
        del dAs, dcs, dmus, dlams, A_plan
    else:
        del outs
    torch.cuda.empty_cache()

    # ---- 3D P1 and P2 Laplacians on the unflattened cube ----------------------
    wl = None
    if any(want(args, k, "laplace") for k in ("laplace3d_fp32", "laplace3d_fp16x2",
                                              "laplace3d_adjoint_fp32",
                                              "laplace3d_adjoint_plan_fp32",
                                              "laplace_p2_3d_fp32", "laplace_p2_3d_fp16x2")):
        wl = meshgen.lap3d(args.n)
        ml = wl.mesh
        El, Nl = ml.n_elements, ml.n_vertices
        # 129 MB per set: enough copies that the cycle exceeds twice the cache
        SL = max(S, -(-2 * MALL_BYTES // forward_bytes(El, Nl, 4, 3, False)) + 1)
        lsets = replicate(torch, dev, (ml.soa(), ml.conn), SL)
        lb = forward_bytes(El, Nl, 4, 3, False)
        # reference at this size: a plain device copy moving the same bytes (half
        # read, half written), over as many buffer pairs as the leg rotates
        lcopy_gbs = copy_gbs
        if want(args, "copy_laplace3d_size", "ref") and (want(args, "laplace3d_fp32", "laplace")
                                                         or want(args, "laplace3d_fp16x2", "laplace")):
            half = lb // 8
            csrc = [torch.ones(half, dtype=torch.float32, device=dev) for _ in range(SL)]
            cdst = [torch.empty_like(x) for x in csrc]
            rc = time_leg([(lambda k=k: cdst[k].copy_(csrc[k])) for k in range(SL)], args.steps,
                          args.warmup, "copy_laplace3d_size")
            lcopy_gbs = 2 * half * 4 / (rc["ms_per_launch"] * 1e-3) / 1e9
            legs["copy_laplace3d_size_reference"] = dict(
                rc, gbs=lcopy_gbs, frac=lcopy_gbs / HBM_PEAK_GBS, traffic_bytes_per_launch=2 * half * 4,
                buffer_sets=SL, note="device copy moving the 3D P1 Laplacian forward's bytes; the "
                "Laplacian forwards' frac_of_measured_copy is taken against it")
            del csrc, cdst
        Al = [torch.empty((El, 4, 4), dtype=torch.float32, device=dev) for _ in range(SL)]
        for prec in ("fp32", "fp16x2"):
            name = f"laplace3d_{prec}"
            if not want(args, name, "laplace"):
                continue
            fns = [(lambda k=k: fei.integrate(lsets[k][0], lsets[k][1], "laplace_p1",
                                              precision=prec, out=Al[k])) for k in range(SL)]
            r = time_leg(fns, args.steps, args.warmup, name)
            legs[name] = rates(r, lb, El, paper_flops(3, 4), lcopy_gbs,
                               stored_traffic(f"laplace_p1_3d_fwd_{prec}"))
        if not args.no_accuracy and "laplace3d_fp32" in legs:
            import oracle
            rng = np.random.Generator(np.random.PCG64(8))
            idx = np.sort(rng.choice(El, 100000, replace=False))
            Ao = oracle.integrate("laplace_p1", ml.coords, ml.conn[idx])
            for prec in ("fp32", "fp16x2"):
                if f"laplace3d_{prec}" in legs:
                    fei.integrate(lsets[0][0], lsets[0][1], "laplace_p1", precision=prec, out=Al[0])
                    As = Al[0][torch.from_numpy(idx).to(dev)].cpu().numpy()
                    acc[f"laplace3d_{prec}"] = dict(error_summary(element_errors(As, Ao)),
                                                    sample="100,000 elements")
        del Al
        # adjoint: single call (atomic scatter) and one-mesh plan
        lab = adjoint_bytes(El, Nl, 4, 3, False)
        dAl_h = meshgen.upstream(El, 4, 1104)
        if want(args, "laplace3d_adjoint_fp32", "laplace") or \
                want(args, "laplace3d_adjoint_plan_fp32", "laplace"):
            dAl = [torch.from_numpy(dAl_h).to(dev) for _ in range(SL)]
            dcl = [torch.zeros((3, Nl), dtype=torch.float32, device=dev) for _ in range(SL)]

            def lacc(name, run):
                if args.no_accuracy:
                    return
                import oracle
                dcl[0].zero_()
                run()
                torch.cuda.synchronize()
                acc[name] = adjoint_accuracy(oracle, ml, "laplace_p1",
                                             dcl[0].cpu().numpy().T.astype(np.float64), dAl_h,
                                             None, None)

            if want(args, "laplace3d_adjoint_fp32", "laplace"):
                fns = [(lambda k=k: fei.integrate_adjoint(lsets[k][0], lsets[k][1], "laplace_p1",
                                                          dAl[k], dcoords=dcl[k]))
                       for k in range(SL)]
                r = time_leg(fns, args.steps, args.warmup, "laplace3d_adjoint_fp32")
                legs["laplace3d_adjoint_fp32"] = rates(
                    r, lab, El, 0, copy_gbs, stored_traffic("laplace_p1_3d_adjoint_fp32"))
                lacc("laplace3d_adjoint_fp32", fns[0])
            if want(args, "laplace3d_adjoint_plan_fp32", "laplace"):
                plans = [fei.Batch([{"form": "laplace_p1", "coords": lsets[k][0],
                                     "conn": lsets[k][1], "dA": dAl[k], "dcoords": dcl[k]}])
                         for k in range(SL)]
                cfg = plans[0].tune(adjoint=True)
                for p in plans[1:]:
                    p.set_config(cfg, adjoint=True)
                r = time_leg([p.run_adjoint for p in plans], args.steps, args.warmup,
                             "laplace3d_adjoint_plan_fp32")
                legs["laplace3d_adjoint_plan_fp32"] = rates(
                    r, lab, El, 0, copy_gbs, stored_traffic("laplace_p1_3d_adjoint_plan_fp32"))
                legs["laplace3d_adjoint_plan_fp32"]["tuned_config"] = cfg
                lacc("laplace3d_adjoint_plan_fp32", plans[0].run_adjoint)
                for p in plans:
                    p.close()
            del dAl, dcl
        # 3D P2 Laplacian (10 x 10 matrices)
        pb = forward_bytes(El, Nl, 10, 3, False)
        SP = max(S, -(-2 * MALL_BYTES // pb) + 1)
        A2 = [torch.empty((El, 10, 10), dtype=torch.float32, device=dev) for _ in range(SP)]
        for prec in ("fp32", "fp16x2"):
            name = f"laplace_p2_3d_{prec}"
            if not want(args, name, "laplace"):
                continue
            fns = [(lambda k=k: fei.integrate(lsets[k % SL][0], lsets[k % SL][1], "laplace_p2",
                                              precision=prec, out=A2[k])) for k in range(SP)]
            r = time_leg(fns, args.steps, args.warmup, name)
            legs[name] = rates(r, pb, El, paper_flops(3, 10), copy_gbs,
                               stored_traffic(f"laplace_p2_3d_fwd_{prec}"))
            if not args.no_accuracy:
                import oracle
                rng = np.random.Generator(np.random.PCG64(9))
                idx = np.sort(rng.choice(El, 50000, replace=False))
                fns[0]()
                As = A2[0][torch.from_numpy(idx).to(dev)].cpu().numpy()
                Ao = oracle.integrate("laplace_p2", ml.coords, ml.conn[idx])
                acc[name] = dict(error_summary(element_errors(As, Ao)), sample="50,000 elements")
        del A2, lsets
        torch.cuda.empty_cache()

    # ---- 2D P1 Laplacian, FP64 coordinates, 8,192 triangles (latency-bound) ----
    if want(args, "laplace2d_f64_latency", "laplace"):
        w2 = meshgen.lap2d(args.n)
        m2 = w2.mesh
        c2 = torch.from_numpy(m2.soa()).to(dev)
        k2 = torch.from_numpy(m2.conn).to(dev)
        A2d = torch.empty((m2.n_elements, 3, 3), dtype=torch.float32, device=dev)
        r = time_leg(lambda: fei.integrate(c2, k2, "laplace_p1", out=A2d), args.steps,
                     args.warmup, "laplace2d_f64_latency")
        b2 = forward_bytes(m2.n_elements, m2.n_vertices, 3, 2, False, coord_bytes=8)
        legs["laplace2d_f64_latency"] = rates(r, b2, m2.n_elements, paper_flops(2, 3))
        legs["laplace2d_f64_latency"].update(
            latency_us_mean=r["kernel_ms_mean"] * 1e3, latency_us_median=r["kernel_ms_median"] * 1e3,
            note="0.46 MB per launch: launch-latency-bound, the GB/s is not a bandwidth figure")
        if not args.no_accuracy:
            import oracle
            Ao = oracle.integrate("laplace_p1", m2.coords, m2.conn)
            acc["laplace2d_f64_latency"] = error_summary(element_errors(A2d.cpu().numpy(), Ao))

    if any(want(args, k, "assembly") for k in ("assembly_elastic_p1_3d", "assembly_laplace_p1_3d",
                                                "coefficient_laplace_p1_3d")):
        assembly_legs(fei, meshgen, dev, args, legs, copy_gbs, acc)

    if want(args, "iso_p2_3d", "forms"):
        iso_leg(fei, meshgen, dev, args, legs, copy_gbs, acc)

    if want(args, "form_elastic_p1_3d", "forms"):
        form_leg(fei, meshgen, dev, args, legs, copy_gbs, acc, S)

    if want(args, "batch", "batch"):
        import oracle
        batch_legs(fei, meshgen, oracle, dev, args, legs, copy_gbs, acc)

    # ---- accuracy of the elasticity forward legs ------------------------------
    need_orc = not args.no_cpu_baseline or not args.no_accuracy
    Ao = None
    if need_orc and any(p in legs for p in ("fp32", "fp16x2", "bf16x2", "bf16x3")):
        import oracle
        A = torch.empty((E, 12, 12), dtype=torch.float32, device=dev)
        outputs = {}
        if not args.no_accuracy:
            c, cn, mu, lam = sets[0]
            for prec in ("fp32", "fp16x2", "bf16x2", "bf16x3"):
                if prec in legs:
                    fei.integrate(c, cn, "elastic_p1", mu, lam, precision=prec, out=A)
                    outputs[prec] = A.cpu().numpy()
        del A
        cores = len(os.sched_getaffinity(0))
        threads = oracle.set_threads(int(os.environ.get("OMP_NUM_THREADS", cores)))
        progress(f"oracle: FP64 integration of {E} elements, {threads} threads")
        t0 = time.perf_counter()
        Ao = oracle.integrate("elastic_p1", m.coords, m.conn, w.mu, w.lam)
        t1 = time.perf_counter()
        for prec, Ag in outputs.items():
            err = element_errors(Ag, Ao)
            acc[prec] = error_summary(err)
            acc[prec]["flattened_max"] = float(err[m.flattened].max())
        # ---- CPU baseline: the FP64 oracle on the same workload -------------
        if not args.no_cpu_baseline:
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
            # one core, on a bounded sample of the same elements
            oracle.set_threads(1)
            n1 = min(E, 200000)
            sub = m.conn[:n1]
            reps1, tot1 = 0, 0.0
            while tot1 < 3.0:
                ta = time.perf_counter()
                oracle.integrate("elastic_p1", m.coords, sub, w.mu[:n1], w.lam[:n1])
                tot1 += time.perf_counter() - ta
                reps1 += 1
            oracle.set_threads(threads)
            result["cpu_baseline_1core"] = {
                "value": reps1 * n1 / tot1, "unit": "element matrices/s", "cores": 1,
                "kind": "oracle",
                "sample": f"{reps1} pass(es) over the first {n1} elements, {tot1:.2f} s wall"}
    result["legs"] = legs
    result["accuracy_vs_oracle"] = acc
    print(json.dumps(result), flush=True)


if __name__ == "__main__":
    main()
