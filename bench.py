#!/usr/bin/env python3
"""Benchmark of the AARMR analysis step on one MI355X.

Headline workload (one "step"): 50 applications of the fine-grid FP64
element-by-element stiffness product y = K(rho~) v (eq. 7's operator with
the Dirichlet identity rows) on the 256x128x128 hex8 cantilever
(4,194,304 elements, 12,830,211 DOFs), whose density is a Gaussian-smoothed
random field (correlation length 8 voxels) mapped to [1e-3, 1].  Two
independent meshes (seeds 3 and 4: moduli, mask, v and y each) alternate,
so the ~490 MB working set exceeds the 256 MB Infinity Cache and the
traffic is HBM traffic.  ``value`` is GDOF/s: 3 n_node x products / s.

``roofline`` is that kernel (HIP events on the library's stream over the
timed region); ``cpu_baseline`` is the CPU FP64 oracle's element-by-element
product on the same grid in the same unit.  Further keys: whole analyses of
the same grid in FP64 and in the FP32-refinement form (solves/s at rel.
residual 1e-8, compliance error against FP64), the 50-cycle AARMR
optimisation loop of the 96x48x48 cantilever, the 64-instance batch and
the served request stream.
"""

from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "EbE K·v GDOF/s; solves/s at 1e-6 rel. compliance; p50/p99 latency vs plain"
HBM_PEAK_GBS = 8000.0

KV_GRID = (256, 128, 128)
# grid levels of the 256x128x128 analyses: 6 (coarsest 8x4x4, 675 DOFs) measured
# fastest, 23.8 / 19.8 ms (FP64 / refinement) against 25.2 / 22.7 ms with 5
# levels (a 4131-DOF coarsest inverse) and 26.2 / 21.5 ms with 7
LEVELS_256 = 6
KV_PER_STEP = 50  # products per timed step (25 per mesh)
NX, NY, NZ = 96, 48, 48
CYCLES, N_ON, NS, NM = 50, 20, 2, 6
VOLFRAC, RMIN, MOVE, CA_TOL = 0.3, 2.0, 0.2, 1e-3


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--loop-steps", type=int, default=3,
                    help="timed runs of the 96x48x48 optimisation loop (extra key)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true",
                    help="skip the comparison run with plain MGCG every cycle")
    ap.add_argument("--kv-launches", type=int, default=200)
    ap.add_argument("--no-precision", action="store_true",
                    help="skip the 256x128x128 FP64 vs refinement-form solve")
    ap.add_argument("--precision-only", action="store_true",
                    help="only the 256x128x128 FP64 vs refinement-form solve")
    ap.add_argument("--no-ca-study", action="store_true",
                    help="skip the bridge loop and the eps / compliance-error relation")
    ap.add_argument("--ca-study-only", action="store_true")
    ap.add_argument("--loop-only", action="store_true",
                    help="only the 96x48x48 optimisation loop (for kernel traces)")
    ap.add_argument("--no-batch", action="store_true", help="skip the 64-instance batch")
    ap.add_argument("--batch-only", action="store_true", help="only the 64-instance batch")
    ap.add_argument("--no-serve", action="store_true", help="skip the serving workload")
    ap.add_argument("--serve-only", action="store_true", help="only the serving workload")
    ap.add_argument("--study", choices=["nsnm", "bridge", "inverter"],
                    help="run a parameter study instead of the benchmark")
    ap.add_argument("--kv-only", action="store_true",
                    help="only the 256x128x128 K.v timing (for hardware-counter runs)")
    ap.add_argument("--kv-sizes", action="store_true",
                    help="only the K.v rate by grid size, 64x32x32 to 704x384x320")
    return ap.parse_args()


def make_loop_state(torch, aarmr, synth):
    prob = synth.cantilever(NX, NY, NZ)
    p = aarmr.default_params(nx=NX, ny=NY, nz=NZ, rmin=RMIN, mg_levels=4, cg_rtol=1e-8,
                             cg_maxit=2000, Ns=NS, Nm=NM, ca_tol=CA_TOL)
    mesh = aarmr.Mesh(p)
    mesh.autotune()  # launch shape of the fine-grid operator, chosen once per mesh
    dev = torch.device("cuda")
    fixed = torch.tensor(aarmr.fixed_dofs_soa(prob, mesh.n_node), dtype=torch.int64, device=dev)
    f = torch.tensor(aarmr.loads_soa(prob, mesh.n_node)[0], dtype=torch.float64, device=dev)
    ones = torch.ones(mesh.n_elem, dtype=torch.float64, device=dev)
    dv = torch.empty_like(ones)
    mesh.filter(ones, dv, mode=1)  # d(volume)/d(design) through eq. (33)
    return mesh, fixed, f, dv


def run_loop(torch, aarmr, mesh, fixed, f, dv, plain=False, record=None, reuse=False):
    """One full optimisation run; returns per-cycle wall times (ms) and paths."""
    dev = f.device
    x = torch.full((mesh.n_elem,), VOLFRAC, dtype=torch.float64, device=dev)
    xn = torch.empty_like(x)
    rp = torch.empty_like(x)
    u = torch.zeros_like(f)
    dc = torch.empty_like(x)
    lat, paths, comp = [], [], []
    fl = aarmr.FILTER_INPUT | (aarmr.REUSE_COARSEST if reuse else 0)
    inv = 0
    for loop in range(1, CYCLES + 1):
        t0 = time.perf_counter()
        if plain or loop <= N_ON:
            flags = fl | aarmr.WARM_START
            if not plain and loop > N_ON - NS:
                flags |= aarmr.RECORD_PARM
            C, st, code = mesh.solve(x, f, fixed, u, dc=dc, flags=flags)
            paths.append("mgcg")
            if record is not None:
                record.append(("mgcg", st.iterations[0], st.fine_sweeps, st.coarsest_inversions))
        else:
            C, st, code = mesh.ca_update(x, f, fixed, u, dc=dc, flags=fl)
            paths.append("ca" if st.accepted[0] else "fallback")
            if record is not None:
                record.append((paths[-1], st.mgcg_iterations[0], st.fine_sweeps, st.eps[0],
                               st.coarsest_inversions))
        inv += st.coarsest_inversions
        t1 = time.perf_counter()
        mesh.oc_update(x, dc, dv, VOLFRAC, MOVE, xn, rp)
        x, xn = xn, x
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        lat.append(((t1 - t0) * 1e3, (t2 - t0) * 1e3))
        comp.append(C[0])
    if record is not None:
        record.append(("coarsest_inversions", inv))
    return lat, paths, comp


def run_opt(torch, aarmr, synth, prob, cycles, volfrac, rmin, levels, n_on=20, ns=2, nm=2,
            ca_tol=1e-3, orth=0, cg_rtol=1e-8, cg_maxit=2000, plain=False, move=0.2):
    """A full optimisation of `prob` (Algorithm 1 unless `plain`: MGCG every
    cycle) from a uniform design; returns the summed analysis time [ms],
    the path of each cycle and the compliance history."""
    dev = torch.device("cuda")
    p = aarmr.default_params(nx=prob.nx, ny=prob.ny, nz=getattr(prob, "nz", 0), rmin=rmin,
                             mg_levels=levels,
                             cg_rtol=cg_rtol, cg_maxit=cg_maxit, Ns=ns, Nm=nm, ca_tol=ca_tol,
                             orth=orth)
    mesh = aarmr.Mesh(p)
    fixed = torch.tensor(aarmr.fixed_dofs_soa(prob, mesh.n_node), dtype=torch.int64, device=dev)
    f = torch.tensor(aarmr.loads_soa(prob, mesh.n_node)[0], dtype=torch.float64, device=dev)
    ones = torch.ones(mesh.n_elem, dtype=torch.float64, device=dev)
    dv = torch.empty_like(ones)
    mesh.filter(ones, dv, mode=1)
    x = torch.full((mesh.n_elem,), volfrac, dtype=torch.float64, device=dev)
    xn, rp = torch.empty_like(x), torch.empty_like(x)
    u = torch.zeros_like(f)
    dc = torch.empty_like(x)
    t_an, paths, comp, its = 0.0, [], [], 0
    fl = aarmr.FILTER_INPUT
    for loop in range(1, cycles + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if plain or loop <= n_on:
            flags = fl | aarmr.WARM_START | (aarmr.RECORD_PARM if not plain and loop > n_on - ns else 0)
            C, st, code = mesh.solve(x, f, fixed, u, dc=dc, flags=flags)
            paths.append("mgcg")
            its += st.iterations[0]
        else:
            C, st, code = mesh.ca_update(x, f, fixed, u, dc=dc, flags=fl)
            paths.append("ca" if st.accepted[0] else "fallback")
            its += st.mgcg_iterations[0]
        t_an += time.perf_counter() - t0
        mesh.oc_update(x, dc, dv, volfrac, move, xn, rp)
        x, xn = xn, x
        comp.append(C[0])
    torch.cuda.synchronize()
    mesh.close()
    return {"analysis_ms": t_an * 1e3, "paths": paths, "compliance": comp, "cg_iterations": its}


def study_ns_nm(torch, aarmr, synth):
    """Section 4.1.1's Ns/Nm design on a 3D grid: the 48x24x24 cantilever,
    60 cycles, volfrac 0.3, r = 2, N_on = 20, eps_tol = 1e-2, SVD basis (eq. 21),
    Ns, Nm in {1, 2, 3, 4, 6}, against MGCG every cycle."""
    prob = synth.cantilever(48, 24, 24)
    kw = dict(cycles=60, volfrac=0.3, rmin=2.0, levels=3)
    ref = run_opt(torch, aarmr, synth, prob, plain=True, **kw)
    c_ref = ref["compliance"][-1]
    rows = []
    for ns in (1, 2, 3, 4, 6):
        for nm in (1, 2, 3, 4, 6):
            r = run_opt(torch, aarmr, synth, prob, ns=ns, nm=nm, ca_tol=1e-2, orth=1, **kw)
            rows.append({"Ns": ns, "Nm": nm, "analysis_ms": round(r["analysis_ms"], 1),
                         "speedup": round(ref["analysis_ms"] / r["analysis_ms"], 3),
                         "mgcg_calls": sum(p != "ca" for p in r["paths"]),
                         "ca_accepted": r["paths"].count("ca"),
                         "end_compliance": r["compliance"][-1],
                         "end_rel_diff": (r["compliance"][-1] - c_ref) / c_ref})
            print(f"[study] Ns={ns} Nm={nm}: {rows[-1]}", file=sys.stderr, flush=True)
    return {"grid": "48x24x24 cantilever", "cycles": 60, "eps_tol": 1e-2,
            "mgcg_every_cycle": {"analysis_ms": round(ref["analysis_ms"], 1),
                                 "end_compliance": c_ref},
            "cases": rows}


def study_bridge(torch, aarmr, synth):
    """Section 4.2.2: the simply supported beam (four bottom corners fixed,
    unit load at the bottom centre) on the paper's four grids, volfrac 0.2,
    N_on = 20, Ns = Nm = 2, MGCG to rel. residual 1e-6 with at most 50
    iterations (the paper's settings), 80 cycles, r = 2; AARMR with eps_tol
    0.5%, 1% and 5% against MGCG every cycle.  Grid levels: 4 where the sizes
    allow (3 for 84x28x56), the paper's 3 would leave a dense coarsest
    operator above 8192 DOFs on the larger grids."""
    out = []
    for dims, lev in (((72, 24, 48), 4), ((84, 28, 56), 3), ((96, 32, 64), 4),
                      ((120, 40, 80), 4)):
        prob = synth.bridge(*dims)
        kw = dict(cycles=80, volfrac=0.2, rmin=2.0, levels=lev, cg_rtol=1e-6, cg_maxit=50)
        ref = run_opt(torch, aarmr, synth, prob, plain=True, **kw)
        row = {"grid": "x".join(map(str, dims)), "levels": lev,
               "mgcg_ms": round(ref["analysis_ms"], 1), "mgcg_end_compliance": ref["compliance"][-1]}
        for tol in (0.005, 0.01, 0.05):
            r = run_opt(torch, aarmr, synth, prob, ns=2, nm=2, ca_tol=tol, **kw)
            row[f"eps_{tol}"] = {"analysis_ms": round(r["analysis_ms"], 1),
                                 "speedup": round(ref["analysis_ms"] / r["analysis_ms"], 3),
                                 "mgcg_calls": sum(p != "ca" for p in r["paths"]),
                                 "end_rel_diff": (r["compliance"][-1] - ref["compliance"][-1])
                                 / ref["compliance"][-1]}
        print(f"[study] bridge {row}", file=sys.stderr, flush=True)
        out.append(row)
    return {"cycles": 80, "Ns": 2, "Nm": 2, "N_on": 20, "rows": out}


def run_mechanism(torch, aarmr, synth, prob, cycles, levels, plain, ca_tol=1e-3, volfrac=0.3,
                  rmin=2.5, move=0.05, n_on=20, ns=2, nm=2):
    """A full displacement-inverter optimisation (Section 4.3): load cases
    input and dummy output, springs, the output displacement's sensitivity
    (AARMR_MUTUAL_SENS; from the reduced model when CA is accepted), OC
    with eta 0.3.  Returns the summed analysis time, paths, the u_out history
    and CG iterations per MGCG call."""
    dev = torch.device("cuda")
    p = aarmr.default_params(nx=prob.nx, ny=prob.ny, nz=0, rmin=rmin, mg_levels=levels,
                             cg_rtol=1e-6, cg_maxit=200, Ns=ns, Nm=nm, ca_tol=ca_tol,
                             n_rhs_max=2, oc_eta=0.3)
    mesh = aarmr.Mesh(p)
    mesh.set_springs(*aarmr.springs_soa(prob, mesh.n_node))
    fixed = torch.tensor(aarmr.fixed_dofs_soa(prob, mesh.n_node), dtype=torch.int64, device=dev)
    f = torch.tensor(np.concatenate(aarmr.loads_soa(prob, mesh.n_node)),
                     dtype=torch.float64, device=dev)
    ones = torch.ones(mesh.n_elem, dtype=torch.float64, device=dev)
    dv = torch.empty_like(ones)
    mesh.filter(ones, dv, mode=1)
    x = torch.full((mesh.n_elem,), volfrac, dtype=torch.float64, device=dev)
    xn, rp = torch.empty_like(x), torch.empty_like(x)
    u = torch.zeros_like(f)
    dc = torch.empty_like(x)
    out_dof = prob.nx  # x DOF of the output node (nx, 0)
    t_an, paths, uout, its, calls = 0.0, [], [], 0, 0
    fl = aarmr.FILTER_INPUT | aarmr.MUTUAL_SENS
    for loop in range(1, cycles + 1):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if plain or loop <= n_on:
            flags = fl | aarmr.WARM_START | (aarmr.RECORD_PARM if not plain and loop > n_on - ns else 0)
            C, st, code = mesh.solve(x, f, fixed, u, dc=dc, flags=flags)
            paths.append("mgcg")
            its += st.iterations[0] + st.iterations[1]
            calls += 2
        else:
            C, st, code = mesh.ca_update(x, f, fixed, u, dc=dc, flags=fl)
            acc = st.accepted[0] and st.accepted[1]
            paths.append("ca" if acc else "fallback")
            for l in range(2):
                if not st.accepted[l]:
                    its += st.mgcg_iterations[l]
                    calls += 1
        t_an += time.perf_counter() - t0
        uout.append(float(u[out_dof]))
        mesh.oc_update(x, dc, dv, volfrac, move, xn, rp)
        x, xn = xn, x
    torch.cuda.synchronize()
    mesh.close()
    return {"analysis_ms": t_an * 1e3, "paths": paths, "u_out": uout,
            "avg_cg_iterations": its / max(calls, 1), "mgcg_solves": calls}


def study_inverter(torch, aarmr, synth, cycles=200):
    """Section 4.3 / Table 1: the displacement inverter on the L-grid 320x160
    and the H-grid 640x320, 200 cycles, volfrac 0.3, N_on = 20, Ns = Nm = 2,
    MGCG to rel. residual 1e-6 with at most 200 iterations, k_in = 1,
    k_out = 0.1; AARMR with eps_tol 0.01% and 0.1% against MGCG every cycle.
    Levels: 4 and 5 (coarsest 1722 DOFs); OC move 0.05, eta 0.3."""
    rows = []
    for dims, lev in (((320, 160), 4), ((640, 320), 5)):
        prob = synth.inverter2d(*dims)
        ref = run_mechanism(torch, aarmr, synth, prob, cycles, lev, plain=True)
        row = {"grid": "x".join(map(str, dims)), "levels": lev,
               "mgcg": {"analysis_ms": round(ref["analysis_ms"], 1),
                        "avg_cg_iterations": round(ref["avg_cg_iterations"], 3),
                        "u_out_end": ref["u_out"][-1]}}
        for tol in (1e-4, 1e-3):
            r = run_mechanism(torch, aarmr, synth, prob, cycles, lev, plain=False, ca_tol=tol)
            row[f"eps_{tol}"] = {"analysis_ms": round(r["analysis_ms"], 1),
                                 "speedup": round(ref["analysis_ms"] / r["analysis_ms"], 3),
                                 "avg_cg_iterations": round(r["avg_cg_iterations"], 3),
                                 "mgcg_solves": r["mgcg_solves"],
                                 "ca_accepted": r["paths"].count("ca"),
                                 "u_out_end": r["u_out"][-1],
                                 "diff_pct": 100.0 * (r["u_out"][-1] - ref["u_out"][-1])
                                 / abs(ref["u_out"][-1])}
        print(f"[study] inverter {row}", file=sys.stderr, flush=True)
        rows.append(row)
    return {"cycles": cycles, "Ns": 2, "Nm": 2, "N_on": 20, "rows": rows}


def kv_event_timing(torch, aarmr, n_launch, sets):
    """Average duration of the fine-grid K.v kernel in the form the solvers
    launch it (input zero on fixed DOFs), HIP events on the stream the
    library launches on (torch's current stream).  `sets` is a list of
    (mesh, v, y) rotated between launches."""
    s = torch.cuda.current_stream()
    fl = aarmr.INPUT_MASKED
    for (m, v, y) in sets:
        m.apply(v, y, flags=fl)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(s)
    for i in range(n_launch):
        m, v, y = sets[i % len(sets)]
        m.apply(v, y, flags=fl)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1) / n_launch  # ms per launch


KV_SIZES = [(64, 32, 32), (96, 48, 48), (128, 64, 64), (192, 96, 96), (256, 128, 128),
            (384, 192, 192), (512, 256, 256), (704, 384, 320)]


def kv_by_size(torch, aarmr, synth, n_launch=100):
    """The fine-grid K.v by grid size, from the launch floor up to the largest
    grid the mesh check accepts: for each size two meshes (i.i.d. density in
    [1e-3, 1], seeds 3 and 4; each with the fewest levels whose coarsest grid
    stays under 8000 DOFs), `n_launch` products alternating between them in
    the solver form, HIP events.  Returns one row per size."""
    rows = []
    for dims in KV_SIZES:
        lev = None
        for L in range(2, 9):
            sc = 2 ** (L - 1)
            if any(d % sc for d in dims):
                break
            c = [d // sc for d in dims]
            if 3 * (c[0] + 1) * (c[1] + 1) * (c[2] + 1) <= 8000:
                lev = L
                break
        sets = []
        for seed in (3, 4):
            prob = synth.cantilever(*dims)
            m = aarmr.Mesh(aarmr.default_params(nx=dims[0], ny=dims[1], nz=dims[2], mg_levels=lev))
            rho = torch.tensor(synth.uniform_iid(*dims, 1e-3, 1.0, seed=seed).ravel(),
                               dtype=torch.float64, device="cuda")
            fx = torch.tensor(aarmr.fixed_dofs_soa(prob, m.n_node), dtype=torch.int64,
                              device="cuda")
            m.setup(rho, fx)
            g = torch.Generator(device="cuda").manual_seed(seed)
            v = torch.randn(3 * m.n_node, dtype=torch.float64, device="cuda", generator=g)
            v[fx] = 0.0
            sets.append((m, v, torch.empty_like(v)))
        ms = kv_event_timing(torch, aarmr, n_launch, sets)
        byts, nn = ebe_bytes(*dims)
        rows.append({"grid": "x".join(map(str, dims)), "levels": lev, "us": round(ms * 1e3, 2),
                     "gdof_s": round(3 * nn / ms / 1e6, 1),
                     "alg_GB_s": round(byts / ms / 1e6, 1),
                     "hbm_frac": round(byts / ms / 1e6 / HBM_PEAK_GBS, 3),
                     "working_set_MB": round(2 * byts / 1e6, 1)})
        print(f"[bench] kv {rows[-1]}", file=sys.stderr, flush=True)
        for m, v, y in sets:
            m.close()
        del sets
        torch.cuda.empty_cache()
    return rows


def pmc_traffic(grid):
    """HBM bytes per launch of the fine-grid K.v kernel on `grid` ("AxBxC")
    from the committed FETCH_SIZE / WRITE_SIZE counter summary (calibrated by
    a 1 GiB copy), or None when the kernel source has changed since the
    counters were taken or no summary exists."""
    import hashlib
    import re

    path = os.path.join(ROOT, "profiles", "ebe_kv_pmc_traffic.txt")
    src = os.path.join(ROOT, "paper_2205_00385_amd", "csrc", "kernels_ebe.hip")
    try:
        text = open(path).read()
        h = hashlib.sha256(open(src, "rb").read()).hexdigest()[:16]
    except OSError:
        return None
    m = re.search(r"sha256\[:16\]=([0-9a-f]{16})", text)
    if not m or m.group(1) != h:
        return None
    m = re.search(r"kv grid=%s .*traffic_bytes=(\d+)" % re.escape(grid), text)
    return int(m.group(1)) if m else None


def ebe_bytes(nx, ny, nz):
    """Algorithmic HBM bytes of one FP64 K.v sweep: read v and write y
    (3 x 8 B per node each), the node's fixed-DOF mask byte, and one
    modulus (8 B) per element."""
    nn = (nx + 1) * (ny + 1) * (nz + 1)
    ne = nx * ny * nz
    return 49 * nn + 8 * ne, nn


def kv_sets(torch, aarmr, synth):
    """Two independent 256x128x128 cantilever meshes (smoothed random fields,
    seeds 3 and 4, in [1e-3, 1]) with their moduli and masks set up and a
    random v (zero on fixed DOFs) and an output y each: ~490 MB together,
    more than the 256 MB Infinity Cache."""
    dev = torch.device("cuda")
    L = KV_GRID
    prob = synth.cantilever(*L)
    sets = []
    for seed in (3, 4):
        p = aarmr.default_params(nx=L[0], ny=L[1], nz=L[2], mg_levels=6)
        m = aarmr.Mesh(p)
        rho = synth.smoothed_field(*L, 8.0, 1e-3, 1.0, seed=seed).ravel()
        fx = torch.tensor(aarmr.fixed_dofs_soa(prob, m.n_node), dtype=torch.int64, device=dev)
        m.setup(torch.tensor(rho, dtype=torch.float64, device=dev), fx)
        nb = 3 * m.n_node
        g = torch.Generator(device=dev)
        g.manual_seed(seed)
        vb = torch.randn(nb, dtype=torch.float64, device=dev, generator=g)
        vb[fx] = 0.0
        sets.append((m, vb, torch.empty(nb, dtype=torch.float64, device=dev)))
    return sets


def kv_roofline(ms, grid, extra=None):
    bb, nnb = ebe_bytes(*grid)
    gb = bb / (ms * 1e-3) / 1e9
    out = {"bound": "hbm", "achieved": round(gb, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
           "frac": round(gb / HBM_PEAK_GBS, 4), "traffic": pmc_traffic("x".join(map(str, grid))),
           "kernel": "k_ebe_z (fine-grid K.v, FP64)", "grid": "x".join(map(str, grid)),
           "ms_per_launch": round(ms, 5), "bytes_per_launch": bb,
           "gdof_s": round(3 * nnb / (ms * 1e-3) / 1e9, 2)}
    if extra:
        out.update(extra)
    return out


def precision_form(torch, aarmr, synth, reps=3):
    """One analysis (setup + MGCG to rel. residual 1e-8, compliance) of the
    256x128x128 cantilever on a smoothed random field (correlation length 8
    voxels, seed 3, mapped to [1e-3, 1]), 6 grid levels (coarsest 8x4x4), in FP64 and in the
    refinement form (FP32 operator sweeps, V-cycle and inner CG; FP64
    residuals, dot accumulation and updates of u).  Median of `reps` timed
    solves after one warm-up solve, each from u = 0."""
    import numpy as np

    dev = torch.device("cuda")
    L = (256, 128, 128)
    prob = synth.cantilever(*L)
    rho = torch.tensor(synth.smoothed_field(*L, 8.0, 1e-3, 1.0, seed=3).ravel(),
                       dtype=torch.float64, device=dev)
    res = {}
    for prec in (aarmr.FP64, aarmr.FP32_REFINE):
        p = aarmr.default_params(nx=L[0], ny=L[1], nz=L[2], mg_levels=LEVELS_256, cg_rtol=1e-8,
                                 cg_maxit=2000, precision=prec)
        m = aarmr.Mesh(p)
        fixed = torch.tensor(aarmr.fixed_dofs_soa(prob, m.n_node), dtype=torch.int64, device=dev)
        f = torch.tensor(np.asarray(aarmr.loads_soa(prob, m.n_node)[0]), dtype=torch.float64,
                         device=dev)
        u = torch.zeros_like(f)
        times = []
        for r in range(reps + 1):
            u.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            C, st, code = m.solve(rho, f, fixed, u)
            dt = time.perf_counter() - t0
            if r > 0:
                times.append(dt)
        res[prec] = {"ms": float(np.median(times)) * 1e3, "C": C[0], "u": u.clone(),
                     "its": int(st.iterations[0]), "rel": float(st.rel_residual[0]),
                     "code": int(code)}
        print(f"[bench] precision form {prec}: {res[prec]['ms']:.2f} ms, "
              f"{res[prec]['its']} its", file=sys.stderr, flush=True)
        m.close()
        del m, u
    a, b = res[aarmr.FP64], res[aarmr.FP32_REFINE]
    du = float(torch.linalg.norm(b["u"] - a["u"]) / torch.linalg.norm(a["u"]))
    return {"workload": "256x128x128 hex8 cantilever, smoothed random field [1e-3, 1], "
                        f"{LEVELS_256} levels, rel. residual 1e-8, one load case",
            "dofs": 3 * (L[0] + 1) * (L[1] + 1) * (L[2] + 1),
            "fp64": {"ms_per_solve": round(a["ms"], 3), "solves_s": round(1e3 / a["ms"], 3),
                     "iterations": a["its"], "rel_residual": a["rel"]},
            "fp32_refine": {"ms_per_solve": round(b["ms"], 3), "solves_s": round(1e3 / b["ms"], 3),
                            "iterations": b["its"], "rel_residual": b["rel"]},
            "speedup": round(a["ms"] / b["ms"], 3),
            "compliance_rel_diff": abs(b["C"] - a["C"]) / abs(a["C"]),
            "u_rel_l2_diff": du,
            "within_1e-6": bool(abs(b["C"] - a["C"]) <= 1e-6 * abs(a["C"]) and du <= 1e-6
                                and a["code"] == 0 and b["code"] == 0)}


def batched_form(torch, aarmr, synth, stream_counts=(1, 4), reps=2):
    """The batch workload: 64 independent cantilevers of uneven cube-ish size
    (each axis from {16, ..., 64}, seed 4000+i, max/min <= 2), each with 4
    load cases (unit -z point loads at seeded x=nx face nodes) and a smoothed
    random density (correlation 4 voxels) in [1e-3, 1]; refinement form,
    4 grid levels, rel. residual 1e-8; each mesh's operator launch shape is
    chosen once by aarmr_autotune.  aarmr_batch_solve over 1 and 4 streams,
    median of `reps` timed runs after a warm-up, each from u = 0."""
    import numpy as np

    dev = torch.device("cuda")
    sizes = synth.batch_sizes(64)
    jobs = []
    for i, (nx, ny, nz) in enumerate(sizes):
        prob = synth.point_loads_on_face(nx, ny, nz, n_case=4, seed=4000 + i)
        p = aarmr.default_params(nx=nx, ny=ny, nz=nz, mg_levels=4, cg_rtol=1e-8, cg_maxit=2000,
                                 n_rhs_max=4, precision=aarmr.FP32_REFINE)
        m = aarmr.Mesh(p)
        f = torch.tensor(np.concatenate([np.asarray(v) for v in aarmr.loads_soa(prob, m.n_node)]),
                         dtype=torch.float64, device=dev)
        rho = torch.tensor(synth.smoothed_field(nx, ny, nz, 4.0, 1e-3, 1.0, seed=4000 + i).ravel(),
                           dtype=torch.float64, device=dev)
        fx = torch.tensor(aarmr.fixed_dofs_soa(prob, m.n_node), dtype=torch.int64, device=dev)
        jobs.append(dict(mesh=m, rho=rho, f=f, fixed=fx, u=torch.zeros_like(f)))
    t_tune = time.perf_counter()
    for jb in jobs:  # launch shapes chosen by the autotuner, once per mesh
        jb["mesh"].autotune()
    t_tune = time.perf_counter() - t_tune
    n_solves = 4 * len(jobs)
    out = {"workload": "64 cantilevers, sizes 16..64 per axis (seeds 4000-4063), 4 point-load "
                       "cases each, refinement form, 4 levels, rel. residual 1e-8",
           "elements": int(sum(a * b * c for a, b, c in sizes)), "solves_per_batch": n_solves,
           "autotune_s": round(t_tune, 3)}
    comp_refine = None
    for ns in stream_counts:
        streams = [torch.cuda.Stream() for _ in range(ns)]
        times = []
        for r in range(reps + 1):
            for jb in jobs:
                jb["u"].zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            comp_refine, items, code = aarmr.batch_solve(jobs, streams)
            dt = time.perf_counter() - t0
            if r > 0:
                times.append(dt)
        ok = code == 0 and all(max(it.stats.rel_residual[l] for l in range(it.n_rhs)) <= 1e-8
                               for it in items)
        T = float(np.median(times))
        out[f"streams_{ns}"] = {"ms_per_batch": round(T * 1e3, 2),
                                "solves_s": round(n_solves / T, 2), "all_converged": bool(ok)}
        print(f"[bench] batch {ns} streams: {T * 1e3:.1f} ms", file=sys.stderr, flush=True)
    for jb in jobs:
        jb["mesh"].close()
    # the same 64 analyses in plain FP64, one after another on one stream
    plain = []
    for jb in jobs:
        m = jb["mesh"]
        p = aarmr.default_params(nx=m.nx, ny=m.ny, nz=m.nz, mg_levels=4, cg_rtol=1e-8,
                                 cg_maxit=2000, n_rhs_max=4, precision=aarmr.FP64)
        m64 = aarmr.Mesh(p)
        m64.autotune()
        plain.append(m64)
    times, comp_plain = [], []
    for r in range(reps + 1):
        for jb in jobs:
            jb["u"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        comp_plain = [m64.solve(jb["rho"], jb["f"], jb["fixed"], jb["u"])[0]
                      for m64, jb in zip(plain, jobs)]
        dt = time.perf_counter() - t0
        if r > 0:
            times.append(dt)
    T = float(np.median(times))
    worst = max(abs(a - b) / abs(b) for ca, cb in zip(comp_refine, comp_plain)
                for a, b in zip(ca, cb))
    out["plain_fp64_one_at_a_time"] = {"ms_per_batch": round(T * 1e3, 2),
                                       "solves_s": round(n_solves / T, 2)}
    # and the FP64 meshes through the batch call on 4 streams: how much of the
    # gain is the concurrency and how much the precision
    jobs64 = [dict(jb, mesh=m64) for m64, jb in zip(plain, jobs)]
    streams = [torch.cuda.Stream() for _ in range(4)]
    times = []
    for r in range(reps + 1):
        for jb in jobs64:
            jb["u"].zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        aarmr.batch_solve(jobs64, streams)
        dt = time.perf_counter() - t0
        if r > 0:
            times.append(dt)
    T = float(np.median(times))
    out["fp64_streams_4"] = {"ms_per_batch": round(T * 1e3, 2), "solves_s": round(n_solves / T, 2)}
    out["compliance_max_rel_diff_vs_plain"] = worst
    out["within_1e-6"] = bool(worst <= 1e-6)
    print(f"[bench] batch plain FP64: {T * 1e3:.1f} ms", file=sys.stderr, flush=True)
    for m64 in plain:
        m64.close()
    return out


def served_form(torch, aarmr, synth, n_requests=40):
    """The serving workload: a Poisson stream (seed 5) of analysis requests on
    grids drawn from {32^3, 48^3, 64^3, 96x48x48, 128^3}, 1-8 load cases each,
    half of them repeats of an earlier design perturbed by w <= 5% (eq. 30).
    Served form: 4 workers, refinement form, resident families with the CA
    reanalysis, HBM budget 80% of free memory.  Plain: one request at a time,
    FP64, same residency and CA.  First both at saturation (every request at
    t = 0), then the served form at 0.5x, 0.8x and 1.0x of its saturation
    rate with real-time arrivals.  Every served compliance is compared with
    the plain FP64 result of the same request."""
    from paper_2205_00385_amd import serve

    free, _ = torch.cuda.mem_get_info()
    budget = int(0.8 * free)
    trace = synth.serve_trace(n_requests, 0.0, seed=5)

    def one(workers, prec, reqs, realtime):
        srv = serve.AnalysisServer(budget, n_workers=workers, precision=prec)
        res = srv.run(reqs, realtime=realtime)
        ev = srv.evictions
        srv.close()
        torch.cuda.empty_cache()
        return res, ev

    plain, _ = one(1, aarmr.FP64, trace, False)
    sat, ev = one(4, aarmr.FP32_REFINE, trace, False)
    worst = max(abs(a - b) / abs(b) for ra, rb in zip(sat, plain)
                for a, b in zip(ra.compliance, rb.compliance))
    ok = sum(all(abs(a - b) <= 1e-6 * abs(b) for a, b in zip(ra.compliance, rb.compliance))
             for ra, rb in zip(sat, plain))
    out = {"workload": f"{n_requests} requests (seed 5), grids 32^3/48^3/64^3/96x48x48/128^3, "
                       "1-8 load cases, 50% perturbed repeats (w <= 5%)",
           "plain_fp64_one_at_a_time": serve.summarize(plain),
           "served_saturation": dict(serve.summarize(sat), evictions=ev),
           "compliance_max_rel_diff_vs_plain": worst,
           "requests_within_1e-6": f"{ok}/{len(sat)}"}
    print(f"[bench] serve saturation: {out['served_saturation']}", file=sys.stderr, flush=True)
    sat_qps = out["served_saturation"]["requests_s"]
    for frac in (0.5, 0.8, 1.0):
        tr = synth.serve_trace(n_requests, frac * sat_qps, seed=5)
        res, ev = one(4, aarmr.FP32_REFINE, tr, True)
        out[f"served_qps_{frac}x"] = dict(serve.summarize(res), qps=round(frac * sat_qps, 3),
                                          evictions=ev)
        print(f"[bench] serve {frac}x: {out[f'served_qps_{frac}x']}", file=sys.stderr, flush=True)
    return out


def cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(sets=None, torch=None, aarmr=None, synth=None, reps=32):
    """The oracle's FP64 element-by-element product (oracle.fem.apply_ebe:
    gather, dense 24x24 element products through BLAS, scatter by bincount)
    on the headline grid, in the headline's unit (GDOF/s): `reps` products on
    the full 256x128x128 grid after one untimed product, with the same
    moduli as the first GPU mesh.  The DOF table is built once, outside the
    timed region, as the GPU mesh builds its own once."""
    import numpy as np

    import synth as _synth
    from oracle import fem

    L = KV_GRID
    nn = (L[0] + 1) * (L[1] + 1) * (L[2] + 1)
    rho = _synth.smoothed_field(*L, 8.0, 1e-3, 1.0, seed=3).ravel()
    E = fem.simp(rho)
    KE = fem.hex8_ke()
    edof = fem.element_dofs_grid(*L)
    v = np.random.default_rng(3).standard_normal(3 * nn)
    fem.apply_ebe(*L, E, KE, v, edof)
    t0 = time.perf_counter()
    for _ in range(reps):
        fem.apply_ebe(*L, E, KE, v, edof)
    dt = time.perf_counter() - t0
    cores = len(os.sched_getaffinity(0)) if hasattr(os, "sched_getaffinity") else os.cpu_count()
    return {"value": round(3 * nn * reps / dt / 1e9, 5), "unit": "GDOF/s", "cores": cores,
            "kind": "oracle", "cpu_model": cpu_model(),
            "sample": f"{reps} FP64 element-by-element products on the full "
                      f"{L[0]}x{L[1]}x{L[2]} grid (oracle.fem.apply_ebe; BLAS on all cores, "
                      f"scatter single-threaded): {dt:.1f} s, {dt / reps * 1e3:.0f} ms per product"}


def reuse_form(torch, aarmr, synth, reps=2, levels=(5, LEVELS_256)):
    """A repeat analysis of the 256x128x128 cantilever (FP64, rel. residual
    1e-8) after a smooth 5% density perturbation of the smoothed random
    field, with a new coarsest inverse (plain) and with the previous design's
    inverse kept (AARMR_REUSE_COARSEST), at each grid depth in `levels`:
    5 levels leave a 4131-DOF coarsest system, 6 levels a 675-DOF one whose
    inversion is cheap.  Each timing is the repeat solve alone, after a solve
    of the unperturbed design, warm-started from its solution; median of
    `reps`."""
    import numpy as np

    dev = torch.device("cuda")
    L = (256, 128, 128)
    prob = synth.cantilever(*L)
    r0 = synth.smoothed_field(*L, 8.0, 1e-3, 1.0, seed=3)
    r1 = synth.smooth_perturb(r0, 0.05, seed=33, sigma=4.0)
    rho0 = torch.tensor(r0.ravel(), dtype=torch.float64, device=dev)
    rho1 = torch.tensor(r1.ravel(), dtype=torch.float64, device=dev)
    res = {"workload": "256x128x128 cantilever, FP64, rel. residual 1e-8: repeat solve "
                       "after a smooth 5% density perturbation"}
    for lev in levels:
        m = aarmr.Mesh(aarmr.default_params(nx=L[0], ny=L[1], nz=L[2], mg_levels=lev,
                                            cg_rtol=1e-8, cg_maxit=2000))
        fixed = torch.tensor(aarmr.fixed_dofs_soa(prob, m.n_node), dtype=torch.int64,
                             device=dev)
        f = torch.tensor(np.asarray(aarmr.loads_soa(prob, m.n_node)[0]), dtype=torch.float64,
                         device=dev)
        u = torch.zeros_like(f)
        out = {}
        for name, fl in (("new_inverse", 0), ("kept_inverse", aarmr.REUSE_COARSEST)):
            times, its, inv, Cs = [], [], [], []
            for r in range(reps + 1):
                u.zero_()
                m.solve(rho0, f, fixed, u, flags=aarmr.REUSE_COARSEST)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                C, st, code = m.solve(rho1, f, fixed, u, flags=fl | aarmr.WARM_START)
                dt = time.perf_counter() - t0
                if r > 0:
                    times.append(dt)
                    its.append(int(st.iterations[0]))
                    inv.append(int(st.coarsest_inversions))
                    Cs.append(C[0])
            out[name] = {"ms": round(float(np.median(times)) * 1e3, 3), "iterations": its,
                         "coarsest_inversions": inv, "compliance": Cs[-1]}
        m.close()
        a, b = out["new_inverse"], out["kept_inverse"]
        out["speedup"] = round(a["ms"] / b["ms"], 3)
        out["compliance_rel_diff"] = (abs(a["compliance"] - b["compliance"])
                                      / abs(a["compliance"]))
        print(f"[bench] repeat solve, {lev} levels: {a['ms']:.2f} / {b['ms']:.2f} ms",
              file=sys.stderr, flush=True)
        res[f"levels_{lev}"] = out
        del m, u
    return res


def ca_fidelity(torch, aarmr, synth):
    """How the eq. (29) residual eps of a reduced-model solution relates to
    its compliance and displacement errors.  The 96x48x48 loop runs its 20
    MGCG cycles (the last two build the PARM, Ns = 2); from that design,
    smooth design perturbations of mean size 1e-4 ... 1e-1 are each analysed
    by one reduced-model step (Nm = 6, accepted whatever eps: eps_tol = 1)
    from the unperturbed design's exact solution, and compared with an FP64
    MGCG solve to rel. residual 1e-10 of the perturbed design."""
    import numpy as np

    dev = torch.device("cuda")
    prob = synth.cantilever(NX, NY, NZ)
    mk = lambda rtol: aarmr.Mesh(aarmr.default_params(
        nx=NX, ny=NY, nz=NZ, rmin=RMIN, mg_levels=4, cg_rtol=rtol, cg_maxit=2000, Ns=NS, Nm=NM,
        ca_tol=1.0))
    mesh, ref = mk(1e-10), mk(1e-10)
    fixed = torch.tensor(aarmr.fixed_dofs_soa(prob, mesh.n_node), dtype=torch.int64, device=dev)
    f = torch.tensor(aarmr.loads_soa(prob, mesh.n_node)[0], dtype=torch.float64, device=dev)
    ones = torch.ones(mesh.n_elem, dtype=torch.float64, device=dev)
    dv = torch.empty_like(ones)
    mesh.filter(ones, dv, mode=1)
    x = torch.full((mesh.n_elem,), VOLFRAC, dtype=torch.float64, device=dev)
    xn, rp = torch.empty_like(x), torch.empty_like(x)
    u, ue = torch.zeros_like(f), torch.zeros_like(f)
    dc = torch.empty_like(x)
    FI = aarmr.FILTER_INPUT
    for loop in range(1, N_ON + 1):
        flags = FI | aarmr.WARM_START | (aarmr.RECORD_PARM if loop > N_ON - NS else 0)
        mesh.solve(x, f, fixed, u, dc=dc, flags=flags)
        if loop < N_ON:
            mesh.oc_update(x, dc, dv, VOLFRAC, MOVE, xn, rp)
            x, xn = xn, x
    x0 = x.cpu().numpy().reshape(NZ, NY, NX)
    rows = []
    for k, amp in enumerate((1e-4, 3e-4, 1e-3, 3e-3, 1e-2, 3e-2, 1e-1)):
        xp = torch.tensor(synth.smooth_perturb(x0, amp, seed=500 + k, sigma=2.0, lo=0.0).ravel(),
                          dtype=torch.float64, device=dev)
        mesh.solve(x, f, fixed, u, flags=FI | aarmr.WARM_START)  # reference state: x0, u(x0)
        C, st, _ = mesh.ca_update(xp, f, fixed, u, flags=FI)
        Ce, _, _ = ref.solve(xp, f, fixed, ue, flags=FI | aarmr.WARM_START)
        rows.append({"perturbation": amp, "eps": float(st.eps[0]),
                     "compliance_rel_err": abs(C[0] - Ce[0]) / abs(Ce[0]),
                     "u_rel_err": float(torch.linalg.norm(u - ue) / torch.linalg.norm(ue)),
                     "rank": int(st.rank[0])})
    torch.cuda.synchronize()
    mesh.close()
    ref.close()
    eps = np.array([r["eps"] for r in rows])
    cerr = np.array([r["compliance_rel_err"] for r in rows])
    order = np.argsort(eps)
    safe = 0.0  # largest eps below which every observed step met the 1e-6 compliance bar
    for i in order:
        if cerr[i] > 1e-6:
            break
        safe = float(eps[i])
    return {"workload": "96x48x48 cantilever: design after 20 MGCG cycles, smooth perturbations, "
                        "one reduced-model step each (Nm = 6, Ns = 2) against FP64 MGCG at 1e-10",
            "steps": rows,
            "max_compliance_err_over_eps2": float((cerr / eps ** 2).max()),
            "eps_meeting_1e-6_compliance": safe}


def bridge_loop(torch, aarmr, synth):
    """Section 4.2.2's simply supported beam on its smallest grid (72x24x48,
    four bottom corners fixed, unit load at the bottom centre), volfrac 0.2,
    80 cycles, r = 2, MGCG to rel. residual 1e-6 with at most 50 iterations
    (the paper's settings), 4 levels; AARMR with N_on = 20, Ns = Nm = 2 and
    eps_tol = 1% against MGCG every cycle (eq. 35's speedup)."""
    prob = synth.bridge(72, 24, 48)
    kw = dict(cycles=80, volfrac=0.2, rmin=2.0, levels=4, cg_rtol=1e-6, cg_maxit=50)
    ref = run_opt(torch, aarmr, synth, prob, plain=True, **kw)
    r = run_opt(torch, aarmr, synth, prob, ns=2, nm=2, ca_tol=0.01, **kw)
    return {"workload": "72x24x48 simply supported beam, 80 cycles, eps_tol 1%, Ns = Nm = 2, "
                        "N_on = 20, MGCG rtol 1e-6 / 50 its, 4 levels",
            "paths": {p: r["paths"].count(p) for p in ("mgcg", "ca", "fallback")},
            "mgcg_analysis_ms": round(ref["analysis_ms"], 1),
            "aarmr_analysis_ms": round(r["analysis_ms"], 1),
            "speedup_eq35": round(ref["analysis_ms"] / r["analysis_ms"], 3),
            "end_compliance_rel_diff": (r["compliance"][-1] - ref["compliance"][-1])
            / ref["compliance"][-1]}


def loop_form(torch, aarmr, synth, steps, warmup, plain=True):
    """The 50-cycle AARMR optimisation loop of the 96x48x48 cantilever
    (Algorithm 1: MGCG for cycles 1..20, then the reduced model with the
    MGCG fallback), `steps` timed runs after `warmup`; optionally the same
    loop with MGCG every cycle (the "plain" comparison of eq. 35)."""
    import numpy as np

    mesh, fixed, f, dv = make_loop_state(torch, aarmr, synth)
    for w in range(warmup):
        run_loop(torch, aarmr, mesh, fixed, f, dv)
    torch.cuda.synchronize()
    lat_all, paths_all, comp_last, record = [], [], None, []
    t0 = time.perf_counter()
    for k in range(steps):
        lat, paths, comp = run_loop(torch, aarmr, mesh, fixed, f, dv,
                                    record=record if k == 0 else None)
        lat_all += lat
        paths_all += paths
        comp_last = comp
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    lat_solve = np.array([a for a, _ in lat_all])
    lat_cycle = np.array([b for _, b in lat_all])
    out = {"workload": "AARMR topology-optimisation loop, 96x48x48 hex8 cantilever, 50 cycles "
                       "(N_on=20, Ns=2, Nm=6, eps_tol=1e-3), MGCG 4 levels rtol 1e-8, filter "
                       "r=2, OC volfrac 0.3",
           "runs": steps, "solves_s": round(CYCLES * steps / T, 3),
           "ms_per_run": round(T * 1e3 / steps, 3),
           "latency_ms": {"analysis_p50": round(float(np.percentile(lat_solve, 50)), 3),
                          "analysis_p99": round(float(np.percentile(lat_solve, 99)), 3),
                          "cycle_p50": round(float(np.percentile(lat_cycle, 50)), 3),
                          "cycle_p99": round(float(np.percentile(lat_cycle, 99)), 3)},
           "paths": {p: paths_all.count(p) // steps for p in ("mgcg", "ca", "fallback")},
           "final_compliance": comp_last[-1]}
    out["coarsest_inversions_per_run"] = record[-1][1] if record else None
    out["cg_iterations_per_run"] = sum(r[1] for r in record[:-1]) if record else None
    if os.environ.get("AARMR_BENCH_TRACE"):
        out["trace_first_run"] = record
    if plain:
        tp = time.perf_counter()
        latp, _, compp = run_loop(torch, aarmr, mesh, fixed, f, dv, plain=True)
        Tp = time.perf_counter() - tp
        out["plain_mgcg"] = {"solves_s": round(CYCLES / Tp, 3),
                             "analysis_p50_ms": round(float(np.median([a for a, _ in latp])), 3),
                             "analysis_p99_ms": round(float(np.percentile([a for a, _ in latp], 99)), 3),
                             "final_compliance": compp[-1],
                             "aarmr_speedup_eq35": round(
                                 sum(a for a, _ in latp) / (sum(a for a, _ in lat_all) / steps), 3)}
    mesh.close()
    return out


def kv_steps(torch, aarmr, sets, n_steps):
    """n_steps steps of KV_PER_STEP products alternating over `sets`, in the
    form the solvers launch them (input zero on fixed DOFs); returns the
    elapsed ms from HIP events recorded on the stream the library launches
    on (torch's current stream)."""
    s = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    fl = aarmr.INPUT_MASKED
    e0.record(s)
    for i in range(n_steps * KV_PER_STEP):
        m, v, y = sets[i % len(sets)]
        m.apply(v, y, flags=fl)
    e1.record(s)
    e1.synchronize()
    return e0.elapsed_time(e1)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the AARMR library runs on one GPU only; --gpus must be 1 "
                                   "(no multi-GPU path is built)"}))
        sys.exit(2)
    import numpy as np
    import torch

    import synth
    from paper_2205_00385_amd import aarmr

    if not torch.cuda.is_available():
        print(json.dumps({"error": "no GPU visible"}))
        sys.exit(2)
    torch.cuda.set_device(0)
    if args.study:
        fn = {"nsnm": study_ns_nm, "bridge": study_bridge, "inverter": study_inverter}[args.study]
        print(json.dumps({f"study_{args.study}": fn(torch, aarmr, synth)}))
        return
    if args.loop_only:
        print(json.dumps({"loop_96x48x48": loop_form(torch, aarmr, synth, args.loop_steps, 1,
                                                     plain=False)}))
        return
    if args.ca_study_only:
        print(json.dumps({"bridge_72x24x48_eps1pct": bridge_loop(torch, aarmr, synth),
                          "ca_fidelity_96x48x48": ca_fidelity(torch, aarmr, synth)}))
        return
    if args.serve_only:
        print(json.dumps({"served_form": served_form(torch, aarmr, synth)}))
        return
    if args.batch_only:
        print(json.dumps({"batched_form_64": batched_form(torch, aarmr, synth)}))
        return
    if args.kv_sizes:
        print(json.dumps({"kv_by_grid_size": kv_by_size(torch, aarmr, synth)}))
        return
    if args.precision_only:
        print(json.dumps({"analysis_256x128x128": precision_form(torch, aarmr, synth)}))
        return
    if args.kv_only:
        # a plain copy of known size (1 GiB read + 1 GiB written, four times the
        # Infinity Cache) first, to calibrate the FETCH_SIZE / WRITE_SIZE
        # counters of a counter run
        a = torch.ones(2 ** 27, dtype=torch.float64, device="cuda")
        b = torch.empty_like(a)
        b.copy_(a)
        torch.cuda.synchronize()
        del a, b

    # ---- headline: FP64 K.v on 256x128x128, two meshes alternating ----
    sets = kv_sets(torch, aarmr, synth)
    nn = sets[0][0].n_node
    print(f"[bench] K.v grid {'x'.join(map(str, KV_GRID))}: {3 * nn} DOFs, two meshes",
          file=sys.stderr, flush=True)
    for (m, v, y) in sets:
        m.apply(v, y, flags=aarmr.INPUT_MASKED)
    if args.warmup:
        kv_steps(torch, aarmr, sets, args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ms_ev = kv_steps(torch, aarmr, sets, args.steps)
    torch.cuda.synchronize()
    T = time.perf_counter() - t0
    n_prod = args.steps * KV_PER_STEP
    ms_launch = ms_ev / n_prod
    print(f"[bench] {n_prod} products: {ms_launch * 1e3:.2f} us each", file=sys.stderr, flush=True)
    roofline = kv_roofline(ms_launch, KV_GRID, {
        "note": "two independent meshes (v, y, moduli, mask) alternate so the working set "
                "exceeds the 256 MB Infinity Cache; achieved = algorithmic bytes (49 B per node "
                "+ 8 B per element) / HIP-event time per launch"})
    out = {
        "metric": METRIC,
        "value": round(3 * nn * n_prod / T / 1e9, 2),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(T * 1e3 / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": "FP64 element-by-element K.v (eq. 7 operator, Dirichlet rows), "
                               "256x128x128 hex8 cantilever, smoothed random density "
                               "[1e-3, 1], two meshes alternating, 50 products per step",
                   "elements": KV_GRID[0] * KV_GRID[1] * KV_GRID[2], "dofs": 3 * nn,
                   "parallelism": "single GPU"},
        "roofline": roofline,
    }
    if args.kv_only:
        print(json.dumps(out), flush=True)
        return
    for (m, _, _) in sets:
        m.close()
    del sets
    torch.cuda.empty_cache()
    extra = {}
    if not args.no_precision:
        extra["analysis_256x128x128"] = precision_form(torch, aarmr, synth)
        torch.cuda.empty_cache()
        extra["repeat_analysis_256x128x128"] = reuse_form(torch, aarmr, synth)
        torch.cuda.empty_cache()
    extra["loop_96x48x48"] = loop_form(torch, aarmr, synth, args.loop_steps, 1,
                                       plain=not args.no_plain)
    if not args.no_ca_study:
        extra["bridge_72x24x48_eps1pct"] = bridge_loop(torch, aarmr, synth)
        extra["ca_fidelity_96x48x48"] = ca_fidelity(torch, aarmr, synth)
        torch.cuda.empty_cache()
    # the same K.v on the loop grid (cache-resident working set: GDOF/s only)
    mesh, fixed, _, _ = make_loop_state(torch, aarmr, synth)
    mesh.setup(torch.full((NX * NY * NZ,), VOLFRAC, dtype=torch.float64, device="cuda"), fixed)
    vr = torch.randn(3 * mesh.n_node, dtype=torch.float64, device="cuda")
    vr[fixed] = 0.0
    ms96 = kv_event_timing(torch, aarmr, args.kv_launches, [(mesh, vr, torch.empty_like(vr))])
    extra["loop_96x48x48"]["kv"] = {"ms_per_launch": round(ms96, 5),
                                    "gdof_s": round(3 * mesh.n_node / (ms96 * 1e-3) / 1e9, 2),
                                    "note": "13 MB working set, resident in the Infinity Cache"}
    mesh.close()
    torch.cuda.empty_cache()
    if not args.no_batch:
        extra["batched_form_64"] = batched_form(torch, aarmr, synth)
        torch.cuda.empty_cache()
    if not args.no_serve:
        extra["served_form"] = served_form(torch, aarmr, synth)
        torch.cuda.empty_cache()
    out.update(extra)
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline()
        gpu = out["value"]
        out["cpu_baseline"]["gpu_over_cpu"] = round(gpu / out["cpu_baseline"]["value"], 1)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
