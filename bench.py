#!/usr/bin/env python3
"""Benchmark of the partial-assembly diffusion apply (FP64) on one MI355X.

Workload (the scale sweep): unit-cube hexahedral lattices sized to ~1e7 dofs for
each order p = 1..8, interior vertices jittered by up to 5% of h (seed 2),
trilinear geometry, coefficient kappa = exp(N(0,1)) i.i.d. per element and
quadrature point (seed 3), Gauss rule with q1d = p + 2, essential dofs on the
whole boundary.  One step = one diffusion apply y = A x at every order of the
sweep; `value` = sum_p ndofs_p / sum_p t_p in GDOF/s (every dof, boundary
included).  The mass apply and Jacobi-PCG time-to-1e-8 are reported beside it.
All inputs are resident in HBM before timing starts.

Prints one JSON line.  --gpus N > 1 is refused: the benchmark measures one GPU (the sharded path is a design only).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, GB/s
FP64_PEAK_TFLOPS = 78.6

METRIC = "PA diffusion apply GDOF/s (p=1–8); CG time-to-1e-8, chosen vs plain FP64"


APPLY_SOURCES = ("paper_1911_09220_amd/csrc/k_apply.hip", "paper_1911_09220_amd/csrc/k_setup.hip",
                 "paper_1911_09220_amd/csrc/device.hpp", "paper_1911_09220_amd/csrc/internal.hpp",
                 "paper_1911_09220_amd/csrc/space.cpp")


def log(msg: str) -> None:
    """Progress line on stderr (the JSON result is the only stdout line)."""
    print("# " + msg, file=sys.stderr, flush=True)


def apply_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in APPLY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def recorded_traffic(p: int):
    """HBM bytes per launch of the p-order diffusion apply from the committed counter record,
    or None when the record was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", f"pa_apply_diffusion_p{p}_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != apply_source_hash():
        return None
    return int(rec["traffic_bytes_per_launch"])


def lattice_size(p: int, target_dofs: float) -> int:
    return max(1, int(round((target_dofs ** (1.0 / 3.0) - 1.0) / p)))


def algorithmic_bytes(kind: str, p: int, ne: int, ndofs: int) -> int:
    """x read + y written + stored D + int32 element->dof map, per apply."""
    q = p + 2
    d_bytes = (48 if kind == "diffusion" else 8) * ne * q ** 3
    return 8 * ndofs + 8 * ndofs + d_bytes + 4 * ne * (p + 1) ** 3


def conv_algorithmic_bytes(p: int, ne: int, ndofs: int) -> int:
    """Convection: x + y + 3 values of alpha adj(J) beta per point + element->dof map."""
    q = p + 2
    return 8 * ndofs + 8 * ndofs + 24 * ne * q ** 3 + 4 * ne * (p + 1) ** 3


def grad_algorithmic_bytes(p: int, ne: int, ndofs: int) -> int:
    """Gradient: x + 3 output components + 9 values of w kappa adj(J)^t per point + map
    (divergence: 3 input components + y, the same count)."""
    q = p + 2
    return 8 * ndofs + 24 * ndofs + 72 * ne * q ** 3 + 4 * ne * (p + 1) ** 3


def elas_algorithmic_bytes(p: int, ne: int, ndofs: int) -> int:
    """Elasticity: 3 input and 3 output components + 11 values per point (J^-1, w det J
    lambda, w det J mu) + element->dof map."""
    q = p + 2
    return 24 * ndofs + 24 * ndofs + 88 * ne * q ** 3 + 4 * ne * (p + 1) ** 3


def geom_algorithmic_bytes(p: int, ne: int, ndofs: int) -> int:
    """Recomputed-geometry diffusion: x + y + w*kappa per point + 8 corner nodes per
    element + int32 element->dof map, per apply."""
    q = p + 2
    return 8 * ndofs + 8 * ndofs + 8 * ne * q ** 3 + 192 * ne + 4 * ne * (p + 1) ** 3


def algorithmic_flops(kind: str, p: int, ne: int) -> int:
    D, Q = p + 1, p + 2
    if kind == "diffusion":
        per = 2 * (2 * (2 * D ** 3 * Q + 3 * D * D * Q * Q + 3 * D * Q ** 3)) + 18 * Q ** 3
    else:
        per = 2 * (2 * (D ** 3 * Q + D * D * Q * Q + D * Q ** 3)) + Q ** 3
    return per * ne


def setup_problem(P, torch, p, target, scatter, renumber=False):
    import synth
    n = lattice_size(p, target)
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    ne = mesh["hex"].shape[0]
    kappa = torch.as_tensor(synth.lognormal_iid(ne, p + 2, 1.0, seed=3), device="cuda")
    S = P.Space(P.Mesh.from_dict(mesh), p, renumber=renumber)
    del mesh
    qd = S.qdata(P.DIFFUSION, coeff=kappa)
    qm = S.qdata(P.MASS, coeff=kappa)
    qg = S.qdata(P.DIFFUSION_GEOM, coeff=kappa)
    # gradient and divergence share their quadrature data (9 values per point)
    qgr = S.qdata(P.GRADIENT, coeff=kappa)
    qdv = qgr
    # linear elasticity with (lambda, mu) = (kappa, kappa / 2) per point
    lm = torch.stack([kappa, 0.5 * kappa], dim=-1).contiguous()
    qel = S.qdata(P.ELASTICITY, coeff=lm)
    del kappa, lm
    # convection with the constant velocity (1, 1/2, 1/4)
    beta = torch.tensor([1.0, 0.5, 0.25], dtype=torch.float64, device="cuda").repeat(ne * (p + 2) ** 3)
    qc = S.qdata(P.CONVECTION, coeff=beta)
    del beta
    gen = torch.Generator(device="cuda")
    gen.manual_seed(100 + p)
    x = torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=gen)
    extra = {"grad": P.Operator(S, P.GRADIENT, qgr, constrained=False),
             "grad_y": torch.empty(3 * S.ndofs, dtype=torch.float64, device="cuda")}
    extra["div"] = P.Operator(S, P.DIVERGENCE, qdv, constrained=False)
    extra["div_x"] = x.repeat(3)
    extra["elas"] = P.Operator(S, P.ELASTICITY, qel)
    extra["elas_x"] = extra["div_x"]
    extra["elas_y"] = torch.empty(3 * S.ndofs, dtype=torch.float64, device="cuda")
    return {
        **extra,
        "p": p, "n": n, "space": S, "ne": S.nelem, "ndofs": S.ndofs,
        "diff": P.Operator(S, P.DIFFUSION, qd, scatter=scatter),
        # the deterministic scatter (element vectors, then a fixed-order gather per dof)
        "diff_evec": P.Operator(S, P.DIFFUSION, qd, scatter="evec"),
        "mass": P.Operator(S, P.MASS, qm, scatter=scatter),
        "geom": P.Operator(S, P.DIFFUSION_GEOM, qg, scatter=scatter),
        "conv": P.Operator(S, P.CONVECTION, qc, scatter=scatter),
        "vec3": P.Operator(S, P.DIFFUSION, qd, vector=True),
        "vec3_y": torch.empty(3 * S.ndofs, dtype=torch.float64, device="cuda"),
        "x": x, "y": torch.empty_like(x),
    }


def time_applies(torch, probs, kind, steps, warmup):
    """Per-order mean apply time (s) from HIP events on the launch stream."""
    stream = torch.cuda.current_stream()
    for pr in probs:
        if kind + "_x" not in pr and kind + "_y" in pr and pr[kind + "_y"].numel() == 3 * pr["ndofs"] \
                and kind == "vec3":
            pr["vec3_x"] = pr["x"].repeat(3)
    for _ in range(warmup):
        for pr in probs:
            pr[kind].apply(pr.get(kind + "_x", pr["x"]), pr.get(kind + "_y", pr["y"]))
    torch.cuda.synchronize()
    evs = [[(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in probs] for _ in range(steps)]
    t0 = time.perf_counter()
    for s in range(steps):
        for i, pr in enumerate(probs):
            evs[s][i][0].record(stream)
            pr[kind].apply(pr.get(kind + "_x", pr["x"]), pr.get(kind + "_y", pr["y"]))
            evs[s][i][1].record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    per = [sum(evs[s][i][0].elapsed_time(evs[s][i][1]) for s in range(steps)) / steps / 1e3
           for i in range(len(probs))]
    return per, wall


def copy_bandwidth(torch, nbytes=4 << 30, reps=10):
    """Device-to-device copy of nbytes (one hipMemcpyAsync per rep through torch's copy_),
    timed with HIP events: the achievable streaming rate of this GPU beside the nominal
    8 TB/s.  Bandwidth counts the bytes read plus the bytes written."""
    src = torch.empty(nbytes, dtype=torch.uint8, device="cuda")
    src.fill_(1)
    dst = torch.empty_like(src)
    dst.copy_(src)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(reps):
        dst.copy_(src)
    e1.record(stream)
    torch.cuda.synchronize()
    t = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    torch.cuda.empty_cache()
    return {"bytes_each_way": nbytes, "ms": round(t * 1e3, 4),
            "GBps_read_plus_write": round(2 * nbytes / t / 1e9, 1), "reps": reps}


def cpu_baseline(orders):
    """The oracle on the host cores: its assembled CSR diffusion matrix (constrained),
    applied by the oracle's C/OpenMP timing variant on reduced lattices of the sweep's
    recipe for p <= 3 (the CSR of higher orders outgrows a bounded sample), and its
    Jacobi-PCG to 1e-8 at p = 3 with the sine load."""
    import numpy as np

    import oracle
    import synth
    from oracle import csr_host, forms
    from oracle.forms import assemble_vector
    t_start = time.perf_counter()
    sizes = {1: 1.25e5, 2: 2.5e5, 3: 2.5e5}
    tot_n, tot_t, parts, t_asm = 0.0, 0.0, [], 0.0
    pcg = None
    for p in [q for q in orders if q in sizes]:
        n = lattice_size(p, sizes[p])
        mesh = synth.hex_lattice(n, 0.05, seed=2)
        kappa = synth.lognormal_iid(mesh["hex"].shape[0], p + 2, 1.0, seed=3)
        ta = time.perf_counter()
        sp = oracle.H1Space(mesh, p)
        K = oracle.assemble(sp, forms.element_stiffness(mesh, p, p + 2, kappa))
        b = assemble_vector(sp, forms.element_load(mesh, p, p + 2, synth.sine_source))
        Kc, bc = oracle.constrain(K, b, sp.boundary)
        t_asm += time.perf_counter() - ta
        H = csr_host.HostCSR(Kc)
        x = np.random.default_rng(p).normal(size=sp.ndofs)
        y = np.empty(sp.ndofs)
        H.matvec(x, y)
        reps, t0 = 0, time.perf_counter()
        while True:
            H.matvec(x, y)
            reps += 1
            el = time.perf_counter() - t0
            if el > 1.0 and reps >= 5:
                break
        t_apply = el / reps
        tot_n += sp.ndofs
        tot_t += t_apply
        parts.append(f"p{p}:{sp.ndofs}dofs:{sp.ndofs / t_apply / 1e9:.4f}GDOF/s")
        if p == 3:
            t0 = time.perf_counter()
            _, its, rel = H.pcg_jacobi(bc, Kc.diagonal(), tol=1e-8)
            pcg = {"order": 3, "ndofs": int(sp.ndofs), "iters": its, "rel_res": rel,
                   "seconds": round(time.perf_counter() - t0, 3)}
        del K, Kc, H
    out = {
        "value": round(tot_n / tot_t / 1e9, 5), "unit": "GDOF/s", "cores": csr_host.threads(),
        "kind": "oracle",
        "sample": ("oracle CSR matvec of the assembled constrained diffusion matrix (C/OpenMP "
                   "timing variant, rows split over the threads), one apply per order, on "
                   "reduced lattices of the sweep's recipe, p <= 3 only: " + ", ".join(parts) +
                   f"; oracle assembly {t_asm:.1f}s; leg total "
                   f"{time.perf_counter() - t_start:.1f}s"),
    }
    if pcg is not None:
        out["jacobi_pcg_time_to_1e-8"] = pcg
    return out


def hcurl_algorithmic_bytes(p: int, ne: int, ndofs: int, nc: int) -> int:
    """H(curl) apply: x + y + nc values per point + the element->dof map with one sign
    byte per element dof (4 + 1 bytes)."""
    q = p + 2
    return 16 * ndofs + 8 * nc * ne * q ** 3 + 5 * ne * 3 * p * (p + 1) ** 2


def bench_hcurl(P, torch, orders, target, steps=10, warmup=2):
    """Definite Maxwell operator (alpha curl-curl + beta mass, lognormal (alpha, beta) per
    quadrature point, tangential essential dofs eliminated) on Nedelec spaces of ~target
    dofs, 5% jitter: apply time per order from HIP events (with its y-init)."""
    import synth
    out = {}
    for p in orders:
        n = max(1, int(round((target / (3.0 * p ** 3)) ** (1.0 / 3.0))))
        mesh = synth.hex_lattice(n, 0.05, seed=2)
        ne = mesh["hex"].shape[0]
        S = P.Space(P.Mesh.from_dict(mesh), p, family="nd")
        del mesh
        q = p + 2
        ab = torch.stack([torch.as_tensor(synth.lognormal_iid(ne, q, 1.0, seed=4), device="cuda"),
                          torch.as_tensor(synth.lognormal_iid(ne, q, 1.0, seed=5), device="cuda")],
                         dim=-1).contiguous()
        op = P.Operator(S, P.HCURL_MAXWELL, S.qdata(P.HCURL_MAXWELL, coeff=ab))
        del ab
        gen = torch.Generator(device="cuda")
        gen.manual_seed(200 + p)
        x = torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=gen)
        y = torch.empty_like(x)
        for _ in range(warmup):
            op.apply(x, y)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            op.apply(x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / steps
        by = hcurl_algorithmic_bytes(p, S.nelem, S.ndofs, 12)
        out[str(p)] = {"ndofs": S.ndofs, "elements": S.nelem, "ms": round(t * 1e3, 4),
                       "gdofs": round(S.ndofs / t / 1e9, 3),
                       "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"hcurl p={p}: {out[str(p)]}")
        del op, x, y, S
        torch.cuda.empty_cache()
    return out


def dg_algorithmic_bytes(p: int, ne: int, ndofs: int, nfaces: int, nbfaces: int) -> int:
    """DG convection: x + y + 3 values per volume point + one value per face point + per
    face its code word (4 bytes) and the slot with its two elements' indices (8 bytes)."""
    q = p + 2
    return 16 * ndofs + 24 * ne * q ** 3 + 8 * (nfaces + nbfaces) * q * q + 12 * (nfaces + nbfaces)


def bench_dg(P, torch, orders, target, steps=10, warmup=2):
    """Upwind DG convection (constant velocity (1, 1/2, 1/4)) on discontinuous spaces of
    ~target dofs, 5% jitter: apply time per order (volume kernel + face kernel + y-init)."""
    import synth
    out = {}
    beta = torch.tensor([1.0, 0.5, 0.25], dtype=torch.float64, device="cuda")
    for p in orders:
        n = max(1, int(round(target ** (1.0 / 3.0) / (p + 1))))
        mesh = synth.hex_lattice(n, 0.05, seed=2)
        S = P.Space(P.Mesh.from_dict(mesh), p, family="l2")
        del mesh
        op = P.Operator(S, P.DG_CONVECTION, S.qdata(P.DG_CONVECTION, coeff=beta), constrained=False)
        gen = torch.Generator(device="cuda")
        gen.manual_seed(300 + p)
        x = torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=gen)
        y = torch.empty_like(x)
        for _ in range(warmup):
            op.apply(x, y)
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(steps):
            op.apply(x, y)
        e1.record(stream)
        torch.cuda.synchronize()
        t = e0.elapsed_time(e1) / 1e3 / steps
        nf = 3 * n * n * (n - 1)
        nb = 6 * n * n
        by = dg_algorithmic_bytes(p, S.nelem, S.ndofs, nf, nb)
        out[str(p)] = {"ndofs": S.ndofs, "elements": S.nelem, "ms": round(t * 1e3, 4),
                       "gdofs": round(S.ndofs / t / 1e9, 3),
                       "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}
        log(f"dg p={p}: {out[str(p)]}")
        del op, x, y, S
        torch.cuda.empty_cache()
    return out


def bench_mixed(P, torch, n=45, p=6, tol=1e-8, tol_hi=1e-10):
    """Quadratic warped mesh: FP64 Jacobi-PCG vs FP32/BF16-inner refinement, at tol and at
    the refinement configuration's own tol_hi; every solution's nodal error against the
    exact solution sin(pi x) sin(pi y) sin(pi z) beside its difference to FP64 PCG."""
    import numpy as np

    import synth
    mesh = synth.q2_warped_lattice(n, 0.05)
    S = P.Space(P.Mesh.from_dict(mesh), p)
    del mesh
    u_exact = torch.as_tensor(synth.sine_solution(S.dof_coords()), device="cuda")
    qd = S.qdata(P.DIFFUSION)
    hi = P.Operator(S, P.DIFFUSION, qd)
    b = S.linear_form(P.SOURCE_SINE)
    diag = hi.diagonal()
    lows = {"fp32": P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32),
            "bf16": P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, P.BF16), qdata_dtype=P.BF16)}
    v = b / b.norm()
    hv = hi.apply(v)
    apply_err = {k: float((lo.apply(v.float()).double() - hv).norm() / hv.norm())
                 for k, lo in lows.items()}
    out = {"ndofs": S.ndofs, "elements": S.nelem, "order": p, "mesh": n,
           "apply_rel_err_vs_fp64_apply": apply_err}

    def nodal_err(x):
        return float((x - u_exact).abs().max())

    for t, key in ((tol, "tol_%.0e" % tol), (tol_hi, "tol_%.0e" % tol_hi)):
        x64, i64 = hi.pcg(b, diag=diag, rel_tol=t, max_iter=40000, history=False)
        res = {"fp64_pcg": {"seconds": round(i64["seconds"], 4), "iters": i64["iters"],
                            "true_rel_res": i64["true_rel_res"],
                            "max_nodal_err_vs_exact": nodal_err(x64)}}
        log(f"mixed p={p} {key}: FP64 PCG {i64['iters']} its {i64['seconds']:.3f} s")
        for name, lo in lows.items():
            modes = (("", True), ("_restart", False)) if t == tol else (("", True),)
            for mode, keep in modes:
                x, info = hi.ir_solve(lo, b, diag=diag, rel_tol=t, inner_rel_tol=1e-2,
                                      max_outer=60, max_inner=40000, keep_direction=keep)
                res[f"ir_{name}{mode}"] = {
                    "seconds": round(info["seconds"], 4), "outer": info["outer"],
                    "inner_iters": info["inner_total"], "rel_res": info["rel_res"],
                    "solution_rel_diff_vs_fp64_pcg": float((x - x64).norm() / x64.norm()),
                    "max_nodal_err_vs_exact": nodal_err(x),
                    "speedup_vs_fp64": round(i64["seconds"] / info["seconds"], 3)}
                log(f"mixed p={p} {key}: IR {name}{mode} {info['outer']} outer "
                    f"{info['inner_total']} inner {info['seconds']:.3f} s")
                del x
        out[key] = res
        del x64
    del lows, hi, qd
    torch.cuda.empty_cache()
    return out


def bench_pmg(P, torch, p=3, target=1e7, tol=1e-8, power_iters=20,
              configs=((2, 10, "arithmetic"), (1, 10, "arithmetic"), (2, 5, "arithmetic"),
                       (2, 20, "arithmetic"), (2, 10, "geometric"))):
    """Order multigrid on the sweep's p-order problem (5% jitter, lognormal kappa per
    point): flexible CG with one V-cycle per iteration against FP64 Jacobi-PCG."""
    import synth
    n = lattice_size(p, target)
    mesh = synth.hex_lattice(n, 0.05, seed=2)
    ne = mesh["hex"].shape[0]
    kappa = torch.as_tensor(synth.lognormal_iid(ne, p + 2, 1.0, seed=3), device="cuda")
    M = P.Mesh.from_dict(mesh)
    del mesh
    orders = [p]
    while orders[-1] > 1:
        orders.append(max(1, orders[-1] // 2))
    means = {"arithmetic": P.MEAN_ARITHMETIC, "geometric": P.MEAN_GEOMETRIC,
             "harmonic": P.MEAN_HARMONIC}
    gen = torch.Generator(device="cuda")
    gen.manual_seed(77)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    spaces = [P.Space(M, q) for q in orders]
    torch.cuda.synchronize()
    t_spaces = time.perf_counter() - t0
    fine = P.Operator(spaces[0], P.DIFFUSION, spaces[0].qdata(P.DIFFUSION, coeff=kappa))
    b = spaces[0].linear_form(P.SOURCE_SINE)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    dfine = fine.diagonal()
    torch.cuda.synchronize()
    t_diag = time.perf_counter() - t0
    xj, ij = fine.pcg(b, diag=dfine, rel_tol=tol, max_iter=20000, history=False)
    out = {"order": p, "orders": orders, "ndofs": spaces[0].ndofs,
           "coarse_ndofs": [S.ndofs for S in spaces[1:]], "elements": spaces[0].nelem,
           "tol": tol, "space_setup_seconds": round(t_spaces, 3),
           "jacobi_pcg": {"iters": ij["iters"], "seconds": round(ij["seconds"], 4),
                          "diag_seconds": round(t_diag, 4), "true_rel_res": ij["true_rel_res"]},
           "runs": []}
    log(f"pmg: Jacobi-PCG {ij['iters']} its {ij['seconds']:.3f} s")
    levels = {}
    for degree, coarse_iters, mean in configs:
        if mean not in levels:
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            ops, diags, lmax = [fine], [dfine], []
            for l, S in enumerate(spaces):
                if l > 0:
                    c = S.coeff_mean(kappa, q1d_in=p + 2, q1d_out=S.p + 2, kind=means[mean])
                    ops.append(P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=c)))
                    diags.append(ops[-1].diagonal())
                v = torch.randn(S.ndofs, dtype=torch.float64, device="cuda", generator=gen)
                lmax.append(ops[l].lambda_max(diags[l], v, power_iters))
            torch.cuda.synchronize()
            levels[mean] = (ops, diags, lmax, time.perf_counter() - t0)
        ops, diags, lmax, t_levels = levels[mean]
        G = P.PMG(ops, diags, lmax, degree=degree, coarse_iters=coarse_iters)
        G.fcg(b, rel_tol=1e-2, max_iter=2, history=False)  # warm-up (workspace, kernels)
        x, info = G.fcg(b, rel_tol=tol, max_iter=1000, history=False)
        run = {"degree": degree, "coarse_iters": coarse_iters, "coarse_coefficient": mean,
               "iters": info["iters"], "seconds": round(info["seconds"], 4),
               "status": info["status"], "true_rel_res": info["true_rel_res"],
               "ms_per_iter": round(1e3 * info["seconds"] / max(1, info["iters"]), 3),
               "speedup_vs_jacobi": round(ij["seconds"] / info["seconds"], 3),
               "level_setup_seconds": round(t_levels, 3),
               "lmax": [round(v, 5) for v in lmax],
               "solution_rel_diff_vs_jacobi": float((x - xj).norm() / xj.norm())}
        out["runs"].append(run)
        log(f"pmg: degree {degree} coarse {coarse_iters} {mean}: {info['iters']} its "
            f"{info['seconds']:.3f} s ({run['speedup_vs_jacobi']}x)")
        del G, x
    best = min(out["runs"], key=lambda r: r["seconds"] if r["status"] == "OK" else 1e9)
    out["best"] = best
    return out


def bench_hpmg(P, torch, p=3, target=1e7, tol=1e-8, power_iters=20, degree=2, coarse_iters=10,
               only=None):
    """Multigrid in the mesh size and the order on a refined mesh: a coarse lattice (5%
    jitter) refined by the library three times (p <= 2) or twice (p >= 3, where the order
    levels already end on a small problem), lognormal kappa per point on the finest
    mesh, order p there.  Flexible CG with one V-cycle per iteration, levels p -> .. -> 1
    on the finest mesh and then one step down in mesh size after another, against the
    order-only V-cycle and FP64 Jacobi-PCG on the same mesh."""
    import synth
    depth = 3 if p <= 2 else 2
    nc = max(1, int(round(lattice_size(p, target) / 2 ** depth)))
    meshes = [P.Mesh.from_dict(synth.hex_lattice(nc, 0.05, seed=2))]
    for _ in range(depth):
        meshes.insert(0, meshes[0].refine())
    M0 = meshes[0]
    orders = [p]
    while orders[-1] > 1:
        orders.append(max(1, orders[-1] // 2))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    S0 = P.Space(M0, p)
    ne = S0.nelem
    kappa = torch.as_tensor(synth.lognormal_iid(ne, p + 2, 1.0, seed=3), device="cuda")
    fine = P.Operator(S0, P.DIFFUSION, S0.qdata(P.DIFFUSION, coeff=kappa))
    b = S0.linear_form(P.SOURCE_SINE)
    dfine = fine.diagonal()
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t0
    xj, ij = fine.pcg(b, diag=dfine, rel_tol=tol, max_iter=20000, history=False)
    log(f"hpmg p={p}: {S0.ndofs} dofs, Jacobi-PCG {ij['iters']} its {ij['seconds']:.3f} s")
    gen = torch.Generator(device="cuda")
    gen.manual_seed(78)
    # for p = 1 the order-only plan is one level: its V-cycle is the coarse PCG alone
    plans = {"order_only": [(0, q) for q in orders]}
    for k in range(1, depth + 1):
        name = f"order_then_{k}_refinement" + ("s" if k > 1 else "")
        plans[name] = [(0, q) for q in orders] + [(m, 1) for m in range(1, k + 1)]
    out = {"order": p, "ndofs": S0.ndofs, "elements": ne,
           "mesh": f"{nc}^3 lattice (5% jitter) refined {depth} times", "tol": tol,
           "degree": degree, "coarse_iters": coarse_iters,
           "setup_seconds": round(t_setup, 3),
           "jacobi_pcg": {"iters": ij["iters"], "seconds": round(ij["seconds"], 4)}, "runs": {}}
    if only:
        plans = {k: v for k, v in plans.items() if k in only}
    for name, plan in plans.items():
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        spaces, ops, diags, lmax, coeffs = [S0], [fine], [dfine], [], [kappa]
        for l, (m, q) in enumerate(plan):
            if l > 0:
                S = P.Space(meshes[m], q)
                prev = spaces[-1]
                qin = plan[l - 1][1] + 2
                if plan[l - 1][0] == m:
                    c = prev.coeff_mean(coeffs[-1], q1d_in=qin, q1d_out=q + 2)
                else:
                    c = prev.coeff_parent_mean(S, coeffs[-1], q1d_in=qin, q1d_out=q + 2)
                spaces.append(S)
                coeffs.append(c)
                ops.append(P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=c)))
                diags.append(ops[-1].diagonal())
            v = torch.randn(spaces[l].ndofs, dtype=torch.float64, device="cuda", generator=gen)
            lmax.append(ops[l].lambda_max(diags[l], v, power_iters))
        torch.cuda.synchronize()
        t_levels = time.perf_counter() - t0
        G = P.PMG(ops, diags, lmax, degree=degree, coarse_iters=coarse_iters)
        G.fcg(b, rel_tol=1e-2, max_iter=2, history=False)  # warm-up (workspace, kernels)
        x, info = G.fcg(b, rel_tol=tol, max_iter=1000, history=False)
        out["runs"][name] = {
            "levels": [["fine" if m == 0 else f"{m} refinement(s) coarser", q] for m, q in plan],
            "level_ndofs": [S.ndofs for S in spaces],
            "iters": info["iters"], "seconds": round(info["seconds"], 4),
            "status": info["status"], "true_rel_res": info["true_rel_res"],
            "ms_per_iter": round(1e3 * info["seconds"] / max(1, info["iters"]), 3),
            "speedup_vs_jacobi": round(ij["seconds"] / info["seconds"], 3),
            "level_setup_seconds": round(t_levels, 3),
            "solution_rel_diff_vs_jacobi": float((x - xj).norm() / xj.norm())}
        log(f"hpmg p={p} {name}: {info['iters']} its {info['seconds']:.3f} s")
        del G, x, spaces[1:], ops[1:], diags[1:], coeffs[1:]
    if "order_only" in out["runs"]:
        base = out["runs"]["order_only"]["seconds"]
        for r in out["runs"].values():
            r["speedup_vs_order_only"] = round(base / r["seconds"], 3)
    return out


# The paper's table of 200 partially assembled CG iterations (2D Poisson, ~1.3M dofs),
# read as seconds: best GPU backend (CEED-CUDA, Quadro GV100) and the 16-core MPI run.
PAPER_2D_SECONDS = {"ceed_cuda_gv100": {1: 0.19, 2: 0.15, 4: 0.12, 8: 0.12},
                    "mpi_16core_xeon6130": {1: 2.72, 2: 1.66, 4: 1.45, 8: 1.44}}


def bench_paper2d(P, torch, orders=(1, 2, 4, 8), ndofs=1.3e6, iters=200, reps=3, applies=20):
    """The paper's experiment shape: 2D Poisson on quadrilaterals, ~1.3M dofs, 200
    unpreconditioned CG iterations with the partially assembled operator, p = 1, 2, 4, 8
    (unit square, 5% jitter, sine right-hand side)."""
    import math
    import synth
    out = {"ndofs_target": ndofs, "iterations": iters, "per_p": {},
           "paper_seconds": PAPER_2D_SECONDS}
    for p in orders:
        n = max(1, int(round((math.sqrt(ndofs) - 1.0) / p)))
        mesh = synth.quad_lattice(n, 0.05, seed=2)
        S = P.Space(P.Mesh.from_dict(mesh), p)
        del mesh
        op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION))
        b = S.linear_form(P.SOURCE_SINE)
        best = None
        for _ in range(reps + 1):  # first call warms up
            x, info = op.pcg(b, rel_tol=0.0, max_iter=iters, precond=P.PRECOND_NONE,
                             check_every=iters, history=False)
            assert info["iters"] == iters
            if best is not None or _ > 0:
                best = info["seconds"] if best is None else min(best, info["seconds"])
        xj, ij = op.pcg(b, rel_tol=0.0, max_iter=iters, check_every=iters, history=False)
        xs = torch.randn(S.ndofs, dtype=torch.float64, device="cuda")
        ys = torch.empty_like(xs)
        op.apply(xs, ys)
        torch.cuda.synchronize()
        a, e = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        a.record()
        for _ in range(applies):
            op.apply(xs, ys)
        e.record()
        torch.cuda.synchronize()
        t_apply = a.elapsed_time(e) / applies / 1e3
        Q = p + 2
        by = 8 * S.ndofs * 2 + 24 * S.nelem * Q * Q + 4 * S.nelem * (p + 1) ** 2
        row = {"n": n, "ndofs": S.ndofs, "elements": S.nelem,
               "cg200_seconds": round(best, 5),
               "gdof_it_per_s": round(S.ndofs * iters / best / 1e9, 3),
               "cg200_jacobi_seconds": round(ij["seconds"], 5),
               "rel_res_after_200": info["rel_res"],
               "apply_ms": round(t_apply * 1e3, 4),
               "apply_gdofs": round(S.ndofs / t_apply / 1e9, 3),
               "apply_hbm_frac": round(by / t_apply / 1e9 / HBM_PEAK_GBS, 4),
               "speedup_vs_paper_ceed_cuda": round(PAPER_2D_SECONDS["ceed_cuda_gv100"][p] / best, 1)}
        out["per_p"][str(p)] = row
        log(f"paper2d p={p}: {S.ndofs} dofs, 200 CG its {best * 1e3:.2f} ms "
            f"(paper CEED-CUDA {PAPER_2D_SECONDS['ceed_cuda_gv100'][p]} s), apply {t_apply * 1e3:.3f} ms")
        del op, S, b, x, xj, xs, ys
    return out


def bench_batched(P, torch, nrhs=16, reps=20, tune_cache=None):
    """32 uneven meshes (1e4..1e6 dofs, p = 2..6), nrhs right-hand sides, one graph launch."""
    import synth
    specs = synth.uneven_mesh_list(32)
    out = {"meshes": len(specs), "nrhs": nrhs}
    ops64, ops32, x64, y64, x32, y32 = [], [], [], [], [], []
    total = 0
    for i, sp in enumerate(specs):
        mesh = synth.hex_lattice(sp["n"], 0.05, seed=sp["mesh_seed"])
        S = P.Space(P.Mesh.from_dict(mesh), sp["p"])
        qd = S.qdata(P.DIFFUSION)
        ops64.append(P.Operator(S, P.DIFFUSION, qd))
        ops32.append(P.Operator(S, P.DIFFUSION, P.lowered_qdata(qd, P.F32), qdata_dtype=P.F32))
        g = torch.Generator(device="cuda")
        g.manual_seed(5000 + i)
        x = torch.randn(S.ndofs, nrhs, dtype=torch.float64, device="cuda", generator=g)
        x64.append(x)
        y64.append(torch.empty_like(x))
        x32.append(x.float())
        y32.append(torch.empty_like(x32[-1]))
        total += S.ndofs
    out["total_dofs"] = total
    flops = sum(algorithmic_flops("diffusion", o.space.p, o.space.nelem) for o in ops64) * nrhs
    out["algorithmic_flops"] = flops
    for name, ops, xs, ys in (("f64", ops64, x64, y64), ("f32", ops32, x32, y32)):
        B = P.Batch(ops, nrhs)
        res = {}
        for mode in ("default", "autotuned"):
            if mode == "autotuned":
                B.autotune(xs, ys, cache_path=tune_cache, reps=5)
            B.apply(xs, ys)
            torch.cuda.synchronize()
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record()
            for _ in range(reps):
                B.apply(xs, ys)
            b.record()
            torch.cuda.synchronize()
            t = a.elapsed_time(b) / reps / 1e3
            res[mode] = {"ms": round(t * 1e3, 4), "gdofs_rhs": round(total * nrhs / t / 1e9, 3)}
        desc = B.describe()
        res["tiles"] = desc["groups"]
        # per order and candidate (5 = FP64 matrix cores), ms of that order's launch
        res["tuning_ms"] = desc["tuning"]
        peak = FP64_PEAK_TFLOPS if name == "f64" else 157.3
        res["vector_or_matrix_peak_frac"] = round(
            flops / (res["autotuned"]["ms"] / 1e3) / 1e12 / peak, 4)
        out[name] = res
        log(f"batched: {name} {res['default']['ms']} ms default, {res['autotuned']['ms']} ms tuned")
    return out


def bench_learned(P, torch, n=64, p=3, fields=20, heldout=10, steps=1500, tol=1e-8,
                  stops=(2, 5, 10, 20, 40, 80, 160, 320, 640)):
    """64^3 p = 3 lattice, GRF lognormal coefficient (contrast 1e3, correlation 0.1): the
    learned element preconditioner is trained on pairs from Jacobi-PCG runs on seeded
    training fields of this mesh, then FCG with it is timed against Jacobi-PCG on held-out
    fields."""
    import synth
    from paper_1911_09220_amd import learned as L
    t0 = time.perf_counter()
    mesh = synth.hex_lattice(n, 0.05, seed=22)
    E = mesh["hex"].shape[0]
    S = P.Space(P.Mesh.from_dict(mesh), p)
    del mesh
    pts = synth.lattice_quadrature_points(n, p + 2)

    def field(seed):
        kappa = synth.grf_lognormal(pts, 0.1, 1e3, seed=seed, device="cuda").reshape(E, -1)
        kappa = kappa.contiguous()
        op = P.Operator(S, P.DIFFUSION, S.qdata(P.DIFFUSION, coeff=kappa))
        return op, op.diagonal(), P.learned_features(S, kappa)

    b = S.linear_form(P.SOURCE_SINE)
    # up to 20 fields every operator stays resident; beyond, the compact store (FP32
    # pairs, one shared operator re-assembled per drawn field) keeps 200 fields in memory
    compact = fields > 20
    samples = L.CompactFields(S) if compact else []
    for f in range(fields):
        if compact:
            kappa = synth.grf_lognormal(pts, 0.1, 1e3, seed=1000 + f,
                                        device="cuda").reshape(E, -1).contiguous()
            samples.add_field(kappa, P.learned_features(S, kappa),
                              lambda op, diag: L.jacobi_pairs(op, b, diag, stops=stops))
        else:
            op, diag, feats = field(1000 + f)
            for r, e in L.jacobi_pairs(op, b, diag, stops=stops):
                samples.append((op, feats, diag, r, e))
        log(f"learned: training field {f + 1}/{fields}, {len(samples)} pairs")
    t_pairs = time.perf_counter() - t0
    net = P.Net(p, hidden=64, max_rows=E, max_train_rows=E)
    net.set_params(L.initial_params(net, seed=23))
    t1 = time.perf_counter()
    losses = L.train(net, samples, steps=steps, lr=2e-3, decay_every=max(1, steps // 3),
                     log_every=max(1, steps // 5), log=log)
    torch.cuda.synchronize()
    t_train = time.perf_counter() - t1
    # ablation: the same basis training with the element features zeroed, so the
    # network's output (the element weights) is one constant vector for every element
    if compact:
        zero = torch.zeros_like(samples.fields[0][1])
        abl_samples = samples.without_features(zero)
    else:
        zero = torch.zeros_like(samples[0][1])
        abl_samples = [(o, zero, d, r, e) for (o, _, d, r, e) in samples]
    net0 = P.Net(p, hidden=64, max_rows=E, max_train_rows=E)
    net0.set_params(L.initial_params(net0, seed=23))
    t2 = time.perf_counter()
    losses0 = L.train(net0, abl_samples, steps=steps, lr=2e-3, decay_every=max(1, steps // 3))
    torch.cuda.synchronize()
    ablation = {"net": net0, "zero": zero, "train_seconds": round(time.perf_counter() - t2, 2),
                "loss_last": float(losses0[-50:].mean())}
    del abl_samples
    del samples
    out = {"order": p, "mesh": n, "ndofs": S.ndofs, "train_fields": fields,
           "pair_stops": list(stops), "train_steps": steps, "pair_seconds": round(t_pairs, 2),
           "train_seconds": round(t_train, 2), "loss_first": float(losses[:50].mean()),
           "loss_last": float(losses[-50:].mean()), "tol": tol, "heldout": []}
    if fields < 200:
        out["train_fields_note"] = (
            f"the learned-preconditioner configuration names 200 training fields; this run "
            f"trains on {fields} (pairs cost {t_pairs / max(1, fields):.2f} s per field); "
            f"--learned-fields 200 runs the full count")
    out["constant_weights"] = {
        "what": "same basis training with the element features zeroed (one weight vector "
                "for every element: the network adds nothing)",
        "train_seconds": ablation["train_seconds"], "loss_last": ablation["loss_last"]}
    for f in range(heldout):
        op, diag, feats = field(2000 + f)
        if f == 0:
            # spread of the network's inputs (the 8 octant log-ratios) over the elements:
            # near zero means the coefficient is nearly constant inside an element
            lr = feats[:, 1:9]
            out["feature_spread"] = {"octant_log_ratio_std": float(lr.std()),
                                     "octant_log_ratio_max_abs": float(lr.abs().max())}
        _, ij = op.pcg(b, diag=diag, rel_tol=tol, max_iter=20000, history=False)
        log(f"learned: held-out field {f}: Jacobi-PCG {ij['iters']} its {ij['seconds']:.3f} s")
        _, il = P.fcg_solve(op, b, diag, net=net, feats=feats, rel_tol=tol, max_iter=20000,
                            history=False)
        out["heldout"].append({
            "field": 2000 + f,
            "jacobi_pcg": {"seconds": round(ij["seconds"], 4), "iters": ij["iters"],
                           "true_rel_res": ij["true_rel_res"]},
            "learned_fcg": {"seconds": round(il["seconds"], 4), "iters": il["iters"],
                            "true_rel_res": il["true_rel_res"], "fell_back": il["fell_back"]},
            "speedup": round(ij["seconds"] / il["seconds"], 3)})
        log(f"learned: held-out field {f}: FCG {il['iters']} its {il['seconds']:.3f} s")
        _, ia = P.fcg_solve(op, b, diag, net=ablation["net"], feats=ablation["zero"],
                            rel_tol=tol, max_iter=20000, history=False)
        out["heldout"][-1]["constant_weights_fcg"] = {
            "seconds": round(ia["seconds"], 4), "iters": ia["iters"],
            "true_rel_res": ia["true_rel_res"], "fell_back": ia["fell_back"]}
        log(f"learned: held-out field {f}: constant-weight FCG {ia['iters']} its "
            f"{ia['seconds']:.3f} s")
        del op, diag, feats
    return out


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--orders", default="1,2,3,4,5,6,7,8")
    ap.add_argument("--target-dofs", type=float, default=1e7)
    ap.add_argument("--scatter", choices=["atomic", "evec"], default="atomic")
    ap.add_argument("--renumber", action="store_true",
                    help="sweep spaces number their dofs by first touch in the device element "
                         "order (PAFEM_SPACE_RENUMBER) instead of vertices, edges, faces, interiors")
    ap.add_argument("--cg-orders", default="1,2,3,4,5,6,7,8",
                    help="orders for the Jacobi-PCG solve ('' = none)")
    ap.add_argument("--geom-cg-orders", default="3",
                    help="orders also solved with the recomputed-geometry operator")
    ap.add_argument("--copy-probe", action="store_true",
                    help="only time the device-to-device copy (for counter calibration)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mass", action="store_true")
    ap.add_argument("--no-geom", action="store_true",
                    help="skip the recomputed-geometry diffusion variant")
    ap.add_argument("--no-conv", action="store_true",
                    help="skip the convection, gradient, divergence and elasticity operators")
    ap.add_argument("--forms", default="mixed,batched,learned,pmg,hpmg,paper2d,hcurl,dg",
                    help="solver forms to measure beside the sweep ('' = none)")
    ap.add_argument("--pmg-orders", default="3,6",
                    help="orders of the sweep problems solved with order multigrid")
    ap.add_argument("--hpmg-orders", default="1,2,3,6",
                    help="orders solved with multigrid in mesh size and order")
    ap.add_argument("--hpmg-plans", default="",
                    help="comma-separated subset of order_only, order_then_1_refinement, "
                         "order_then_2_refinements, order_then_3_refinements ('' = all)")
    ap.add_argument("--learned-fields", type=int, default=20)
    ap.add_argument("--learned-steps", type=int, default=1500)
    args = ap.parse_args()

    if args.gpus != 1:
        print(json.dumps({"error": "the benchmark runs on one GPU; the multi-GPU path is not built, so --gpus must be 1",
                          "n_gpus": args.gpus}))
        sys.exit(2)

    import torch

    from paper_1911_09220_amd import pafem as P
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.copy_probe:
        print(json.dumps({"copy": copy_bandwidth(torch)}), flush=True)
        return
    copy = copy_bandwidth(torch)
    log(f"device copy {copy['GBps_read_plus_write']} GB/s (read + write)")
    orders = [int(v) for v in args.orders.split(",") if v]
    t_setup = time.perf_counter()
    probs = []
    for p in orders:
        probs.append(setup_problem(P, torch, p, args.target_dofs, args.scatter, args.renumber))
        print(f"# setup p={p}: {probs[-1]['ndofs']} dofs, {probs[-1]['ne']} elements",
              file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    t_setup = time.perf_counter() - t_setup

    per, wall = time_applies(torch, probs, "diff", args.steps, args.warmup)
    total_dofs = sum(pr["ndofs"] for pr in probs)
    step_s = sum(per)
    value = total_dofs / step_s / 1e9
    per_p = {}
    for pr, t in zip(probs, per):
        by = algorithmic_bytes("diffusion", pr["p"], pr["ne"], pr["ndofs"])
        fl = algorithmic_flops("diffusion", pr["p"], pr["ne"])
        per_p[str(pr["p"])] = {
            "ndofs": pr["ndofs"], "elements": pr["ne"], "ms": round(t * 1e3, 4),
            "gdofs": round(pr["ndofs"] / t / 1e9, 3),
            "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4),
            "fp64_frac": round(fl / t / 1e12 / FP64_PEAK_TFLOPS, 4),
        }
    mass = {}
    if not args.no_mass:
        mper, _ = time_applies(torch, probs, "mass", max(3, args.steps // 2), 1)
        for pr, t in zip(probs, mper):
            by = algorithmic_bytes("mass", pr["p"], pr["ne"], pr["ndofs"])
            mass[str(pr["p"])] = {"ms": round(t * 1e3, 4), "gdofs": round(pr["ndofs"] / t / 1e9, 3),
                                  "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}

    evec = {}
    if not args.no_mass:
        eper, _ = time_applies(torch, probs, "diff_evec", max(3, args.steps // 2), 1)
        for pr, t, ta in zip(probs, eper, per):
            evec[str(pr["p"])] = {"ms": round(t * 1e3, 4), "gdofs": round(pr["ndofs"] / t / 1e9, 3),
                                  "time_vs_atomic": round(t / ta, 3)}

    geom = {}
    if not args.no_geom:
        gper, _ = time_applies(torch, probs, "geom", max(3, args.steps // 2), 1)
        for pr, t, td in zip(probs, gper, per):
            by = geom_algorithmic_bytes(pr["p"], pr["ne"], pr["ndofs"])
            geom[str(pr["p"])] = {"ms": round(t * 1e3, 4), "gdofs": round(pr["ndofs"] / t / 1e9, 3),
                                  "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4),
                                  "speedup_vs_stored": round(td / t, 3)}

    conv = {}
    if not args.no_conv:
        cper, _ = time_applies(torch, probs, "conv", max(3, args.steps // 2), 1)
        for pr, t in zip(probs, cper):
            by = conv_algorithmic_bytes(pr["p"], pr["ne"], pr["ndofs"])
            conv[str(pr["p"])] = {"ms": round(t * 1e3, 4), "gdofs": round(pr["ndofs"] / t / 1e9, 3),
                                  "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}

    vec3 = {}
    if not args.no_conv:
        vper, _ = time_applies(torch, probs, "vec3", max(3, args.steps // 2), 1)
        for pr, t, td in zip(probs, vper, per):
            vec3[str(pr["p"])] = {"ms": round(t * 1e3, 4),
                                  "gdofs_per_component": round(3 * pr["ndofs"] / t / 1e9, 3),
                                  "speedup_vs_3_scalar_applies": round(3 * td / t, 3)}
        for pr in probs:
            pr.pop("vec3_x", None)

    grad = {}
    gprobs = [pr for pr in probs if "grad" in pr]
    if not args.no_conv and gprobs:
        gper2, _ = time_applies(torch, gprobs, "grad", max(3, args.steps // 2), 1)
        for pr, t in zip(gprobs, gper2):
            by = grad_algorithmic_bytes(pr["p"], pr["ne"], pr["ndofs"])
            grad[str(pr["p"])] = {"ms": round(t * 1e3, 4), "gdofs": round(pr["ndofs"] / t / 1e9, 3),
                                  "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}

    div = {}
    if not args.no_conv:
        dper, _ = time_applies(torch, probs, "div", max(3, args.steps // 2), 1)
        for pr, t in zip(probs, dper):
            by = grad_algorithmic_bytes(pr["p"], pr["ne"], pr["ndofs"])
            div[str(pr["p"])] = {"ms": round(t * 1e3, 4), "gdofs": round(pr["ndofs"] / t / 1e9, 3),
                                 "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}

    elas = {}
    if not args.no_conv:
        eper, _ = time_applies(torch, probs, "elas", max(3, args.steps // 2), 1)
        for pr, t in zip(probs, eper):
            by = elas_algorithmic_bytes(pr["p"], pr["ne"], pr["ndofs"])
            elas[str(pr["p"])] = {"ms": round(t * 1e3, 4),
                                  "gdofs": round(3 * pr["ndofs"] / t / 1e9, 3),
                                  "hbm_frac": round(by / t / 1e9 / HBM_PEAK_GBS, 4)}

    # dominant kernel: the order whose apply takes the longest
    k = max(range(len(probs)), key=lambda i: per[i])
    dom = probs[k]
    by = algorithmic_bytes("diffusion", dom["p"], dom["ne"], dom["ndofs"])
    achieved = by / per[k] / 1e9
    roofline = {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                "traffic": recorded_traffic(dom["p"]), "source_hash": apply_source_hash(),
                "kernel": f"pa_apply_kernel diffusion p={dom['p']} q1d={dom['p'] + 2} f64 "
                          f"({args.scatter} scatter, with its y-init kernel)",
                "bytes_per_launch": by,
                "measured_copy_GBps": copy["GBps_read_plus_write"],
                "frac_of_measured_copy": round(achieved / copy["GBps_read_plus_write"], 4)}

    cg = {}
    for p in [int(v) for v in args.cg_orders.split(",") if v]:
        pr = next((q for q in probs if q["p"] == p), None)
        if pr is None:
            continue
        b = pr["space"].linear_form(P.SOURCE_SINE)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        diag = pr["diff"].diagonal()
        torch.cuda.synchronize()
        t_diag = time.perf_counter() - t0
        xs, info = pr["diff"].pcg(b, diag=diag, rel_tol=1e-8, max_iter=20000, history=False)
        cg[str(p)] = {"solver": "jacobi-pcg f64", "iters": info["iters"],
                      "seconds": round(info["seconds"], 4), "status": info["status"],
                      "true_rel_res": info["true_rel_res"], "diag_seconds": round(t_diag, 4),
                      "ms_per_iter": round(1e3 * info["seconds"] / max(1, info["iters"]), 4)}
        if not args.no_geom and str(p) in args.geom_cg_orders.split(","):
            # same solve with the recomputed-geometry operator (diagonal of the stored one)
            xg, gi = pr["geom"].pcg(b, diag=diag, rel_tol=1e-8, max_iter=20000, history=False)
            cg[str(p)]["recomputed_geometry"] = {
                "iters": gi["iters"], "seconds": round(gi["seconds"], 4), "status": gi["status"],
                "true_rel_res": gi["true_rel_res"],
                "ms_per_iter": round(1e3 * gi["seconds"] / max(1, gi["iters"]), 4),
                "rel_diff_vs_stored": float((xg - xs).norm() / xs.norm())}
            del xg
        del xs, b, diag

    out = {
        "metric": METRIC, "value": round(value, 4), "unit": "GDOF/s", "n_gpus": 1,
        "steps": args.steps, "warmup": args.warmup, "ms_per_step": round(step_s * 1e3, 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"scale sweep: unit-cube hex lattices of ~{args.target_dofs:.0e} "
                               f"dofs for p={args.orders}, 5% vertex jitter, lognormal kappa "
                               f"(sigma=1) per quadrature point, q1d=p+2, Dirichlet boundary",
                   "orders": orders, "scatter": args.scatter,
                   "dof_numbering": "first touch in Morton element order" if args.renumber
                   else "vertices, edges, faces, interiors", "per_p": per_p,
                   "mass_apply": mass, "deterministic_scatter_apply": evec,
                   "recomputed_geometry_apply": geom,
                   "convection_apply": conv, "gradient_apply": grad,
                   "divergence_apply": div, "elasticity_apply": elas,
                   "vector_diffusion_apply": vec3, "setup_seconds": round(t_setup, 1),
                   "timed_wall_seconds": round(wall, 4)},
        "roofline": roofline,
        "diffusion_hbm_frac_by_p": {k: v["hbm_frac"] for k, v in per_p.items()},
        "diffusion_frac_of_copy_by_p": {
            k: round(v["hbm_frac"] * HBM_PEAK_GBS / copy["GBps_read_plus_write"], 4)
            for k, v in per_p.items()},
        "device_copy": copy,
        "device": {"name": torch.cuda.get_device_name(0),
                   "arch": getattr(torch.cuda.get_device_properties(0), "gcnArchName", None)},
        "cg_time_to_1e-8": cg,
    }
    forms = [f for f in args.forms.split(",") if f]
    # free the sweep's device memory before the solver forms
    dom = pr = None
    probs.clear()
    torch.cuda.synchronize()
    torch.cuda.empty_cache()
    if "mixed" in forms:
        log("mixed precision")
        out["mixed_precision"] = bench_mixed(P, torch)
        # the same refinement where the apply is bound by HBM: p = 3, ~2e7 dofs
        out["mixed_precision_p3"] = bench_mixed(P, torch, n=90, p=3)
    if "batched" in forms:
        log("batched")
        out["batched"] = bench_batched(P, torch)
    if "pmg" in forms:
        out["pmg"] = {}
        for p in [int(v) for v in args.pmg_orders.split(",") if v]:
            log(f"pmg p={p}")
            out["pmg"][str(p)] = bench_pmg(P, torch, p=p, target=args.target_dofs)
    if "hpmg" in forms:
        out["hpmg"] = {}
        for p in [int(v) for v in args.hpmg_orders.split(",") if v]:
            out["hpmg"][str(p)] = bench_hpmg(P, torch, p=p, target=args.target_dofs,
                                             only=[v for v in args.hpmg_plans.split(",") if v])
    if "hcurl" in forms:
        log("hcurl")
        out["hcurl_maxwell_apply"] = bench_hcurl(P, torch, orders, args.target_dofs)
    if "dg" in forms:
        log("dg")
        out["dg_convection_apply"] = bench_dg(P, torch, orders, args.target_dofs)
    if "paper2d" in forms:
        log("paper2d")
        out["paper_2d_cg200"] = bench_paper2d(P, torch)
    if "learned" in forms:
        log("learned")
        out["learned"] = bench_learned(P, torch, fields=args.learned_fields,
                                       steps=args.learned_steps)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(orders)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
