#!/usr/bin/env python
"""Training throughput of the PNA GCNN hot path on one MI355X.

One step = CSR build + forward of every layer + pooling/head/loss + backward
of every layer + AdamW, over one packed batch already resident in HBM
(6 PNA layers, H = 128, 128 synthetic molecules of 10-60 atoms, FP32).
Prints one JSON line.  The BF16 variant of the same step is timed beside it
and, with the serving loop built, p50/p99 latency at a fixed request rate.
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

HBM_PEAK_GBS = 8000.0
FP32_PEAK_TFLOPS = 157.3
BF16_PEAK_TFLOPS = 2500.0


def _log(msg):
    print(msg, file=sys.stderr, flush=True)


# Counter-derived HBM traffic per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE,
# scaled by a plain copy kernel), kept as short text summaries in profiles/.
# Each names a digest of the file that defines the kernel (and its tile
# header); a summary taken before that source changed no longer describes the
# kernel and is not used.
UPDATE_GEMM_TRAFFIC = ("update_gemm_c1_fp32_traffic.txt",
                       ["csrc/gemm_ntb.hip", "csrc/mfma_tile.hpp"])
# per launch site of the C1 FP32 step (the headline's dominant site is
# looked up here)
SITE_TRAFFIC = {
    "update_gemm": UPDATE_GEMM_TRAFFIC,
    "update_wgrad": ("update_wgrad_c1_fp32_traffic.txt",
                     ["csrc/gemm_tn.hip", "csrc/mfma_tile.hpp"]),
    "aggregate_bwd": ("aggregate_bwd_c1_fp32_traffic.txt",
                      ["csrc/agg_fused.hip", "csrc/agg_msg.hpp", "csrc/mfma_tile.hpp"]),
    "message_wgrad": ("message_wgrad_c1_fp32_traffic.txt",
                      ["csrc/gemm_tn.hip", "csrc/mfma_tile.hpp"]),
    "agg_input_gemm": ("agg_input_gemm_c1_fp32_traffic.txt",
                       ["csrc/gemm_nt.hip", "csrc/mfma_tile.hpp"]),
}
AGGREGATE_TRAFFIC = {
    "aggregate": ("aggregate_c3_traffic.txt", ["csrc/aggregate.hip", "csrc/agg_msg.hpp"]),
    "aggregate_bwd": ("aggregate_bwd_c3_traffic.txt",
                      ["csrc/agg_fused.hip", "csrc/agg_msg.hpp", "csrc/mfma_tile.hpp"]),
}


def measured_traffic(name, sources):
    """Bytes per launch from a committed counter summary, or None when there is
    none or the kernel's sources changed since the counters were taken."""
    from paper_2207_11333_amd import profile_summary as ps
    path = os.path.join(ROOT, "profiles", name)
    if not os.path.exists(path):
        return None
    info = ps.read_summary(path)
    if info.get("sources_sha256") != ps.sources_digest(sources):
        return None
    try:
        return float(info["traffic_bytes_per_launch"])
    except (KeyError, ValueError):
        return None


# Launch sites of the PNA training step timed by the library's event pairs
# (kernel alone for the GEMM and aggregation sites), the kernel each one
# runs (as named in the rocprofv3 summaries) and what bounds it.
# Layers after the first run the message and update linears in the LDS-DMA
# form (k_gemm_ntb: FP32 on the inputs, BF16 on operand copies), FP32 also the
# layer-input gradient; the first layer and the other BF16 sites the
# register-staged kernel.  BF16 weight gradients run k_gemm_tn_tr.
SITES = {
    "message_gemm": ("S1 message linear",
                     "k_gemm_nt<P, 64, 128, *, 2, 4, *> | k_gemm_ntb<P, *, *, 2, 4, 2>", "mfma"),
    "aggregate": ("S2 aggregation", "k_aggregate<1>", "hbm"),
    "update_gemm": ("S3 update linear",
                    "k_gemm_nt<P, 64, 128, *, 1, 4, *> | k_gemm_ntb<P, *, *, 2, 4, 1>", "mfma"),
    "update_wgrad": ("S6 update weight gradient", "k_gemm_tn<P, 64, 64, 1> | k_gemm_tn_tr<1, *>",
                     "mfma"),
    "agg_input_gemm": ("S6 aggregate-input gradient", "k_gemm_nt<P, 64, 128, *, 3, 4, *>", "mfma"),
    # by degree bucket dA is formed inside the adjoint (one fused kernel, dA
    # not stored) and the S6 aggregate-input GEMM site has no launches
    "aggregate_bwd": ("S6 dA + S7 aggregation adjoint, fused", "k_agg_bwd_fused<P, 1, *>", "hbm"),
    "input_gemm": ("S6+S8 layer-input gradient",
                   "k_gemm_nt<P, 64, 128, *, 4, 4, *> | k_gemm_ntb<0, 64, 64, 2, 4, 4>", "mfma"),
    "message_wgrad": ("S8 message weight gradient", "k_gemm_tn<P, 64, 64, 2> | k_gemm_tn_tr<2, *>",
                      "mfma"),
}


def site_work(site, w, N, E):
    """Algorithmic work of one launch of a site (FLOPs for the linears, bytes
    for the aggregations), averaged over the launches of one step, and the
    launches per step.  The linears count the least work the method needs:
    the decomposed message linear [N, F] x [F, 2H], and the update linear by
    degree bucket, [N, F + 4H] x [F + 4H, H] (the degree scalers fold into one
    weight per degree), F = 9 real input features in layer 0 and H after."""
    H, L, Fe = w.hidden, w.num_layers, w.edge_feat
    Fs = [9] + [H] * (L - 1)
    rec = 2 if w.recompute else 1
    if site == "message_gemm":
        return sum(2.0 * N * F * 2 * H for F in Fs) / L, rec * L
    if site == "update_gemm":
        return sum(2.0 * N * (F + 4 * H) * H for F in Fs) / L, L
    if site == "update_wgrad":
        return sum(2.0 * N * H * (F + 4 * H) for F in Fs) / L, L
    if site == "agg_input_gemm":
        return 2.0 * N * H * 4 * H, L
    if site == "input_gemm":
        return 2.0 * N * 3 * H * H, L - 1
    if site == "message_wgrad":
        return sum(2.0 * N * 2 * H * F for F in Fs) / L, L
    if site == "aggregate":
        return float(aggregate_bytes(N, E, H, Fe)), rec * L
    if site == "aggregate_bwd":
        return float(aggregate_bwd_bytes(N, E, H, Fe, fused=True)), L
    raise KeyError(site)


def time_sites(m, step, steps, w, N, E, sites=tuple(SITES)):
    """Per launch site: average kernel duration over `steps` further steps and
    the roofline figures."""
    import torch
    bf16 = w.precision == 1
    out = {}
    for site in sites:
        m.timer_start(site, steps * 2 * w.num_layers + 16)
        torch.cuda.synchronize()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        ms, n = m.timer_read()
        if n == 0:
            continue
        work, per_step = site_work(site, w, N, E)
        avg = ms / 1e3 / n
        what, kern, bound = SITES[site]
        if bound == "hbm":
            ach, peak, unit = work / avg / 1e9, HBM_PEAK_GBS, "GB/s"
        else:
            peak = BF16_PEAK_TFLOPS if bf16 else FP32_PEAK_TFLOPS
            ach, unit = work / avg / 1e12, "TFLOP/s"
        out[site] = {"step": what, "kernel": kern.replace("<P,", f"<{w.precision},"),
                     "bound": bound, "avg_us": avg * 1e6, "launches": n,
                     "launches_per_step": per_step, "us_per_step": avg * 1e6 * per_step,
                     ("bytes_per_launch" if bound == "hbm" else "flops_per_launch"): work,
                     "achieved": ach, "peak": peak, "unit": unit, "frac": ach / peak}
    return out


def dominant_roofline(sites):
    """The roofline object of the site with the most kernel time per step."""
    name = max(sites, key=lambda k: sites[k]["us_per_step"])
    r = dict(sites[name])
    r["site"] = name
    r["traffic"] = measured_traffic(*SITE_TRAFFIC[name]) if name in SITE_TRAFFIC else None
    return r


def phase_split(m, step_parts, steps):
    """Mean time per step of the CSR build (S0, its own event pair), the rest
    of the forward pass, the backward pass and the AdamW step (event pairs on
    the caller's stream between the calls)."""
    import torch
    fwd, bwd, opt = step_parts
    evs = [[torch.cuda.Event(enable_timing=True) for _ in range(4)] for _ in range(steps)]
    m.timer_start("csr", steps + 4)
    torch.cuda.synchronize()
    for e in evs:
        e[0].record()
        fwd()
        e[1].record()
        bwd()
        e[2].record()
        opt()
        e[3].record()
    torch.cuda.synchronize()
    s0_ms, n = m.timer_read()
    s0 = s0_ms / max(1, n)
    mean = lambda a, b: sum(e[a].elapsed_time(e[b]) for e in evs) / steps
    return {"s0_csr_ms": s0, "forward_ms": mean(0, 1) - s0, "backward_ms": mean(1, 2),
            "adamw_ms": mean(2, 3)}


def train_rate(workload, steps, warmup, sites=False, phases=False):
    import torch
    from paper_2207_11333_amd import hgnn
    b = workload.batch()
    m = hgnn.Model(workload.num_layers, workload.hidden, 9, workload.edge_feat, 4,
                   workload.precision, workload.recompute, workload.delta)
    m.set_params(workload.params())
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    loss = torch.empty(1, device="cuda")

    def step():
        m.forward(db, pred, loss)
        m.backward()
        m.adam_step(lr=1e-3)

    m.forward(db, pred, loss, validate=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"graphs_per_s": b.num_graphs * steps / dt, "ms_per_step": 1e3 * dt / steps,
           "B": b.num_graphs, "N": b.num_nodes, "E": b.num_edges,
           "loss": float(loss.item())}
    # the further passes below are timed separately and leave the figures
    # above untouched
    if sites:
        out["sites"] = time_sites(m, step, max(4, min(steps, 20)), workload, b.num_nodes,
                                  b.num_edges)
    if phases:
        out["phases"] = phase_split(m, (lambda: m.forward(db, pred, loss), m.backward,
                                        lambda: m.adam_step(lr=1e-3)), max(4, min(steps, 50)))
    m.close()
    return out


def train_rate_graph(workload, steps, warmup):
    """Same step, captured once as a HIP graph and replayed."""
    import torch
    from paper_2207_11333_amd import hgnn
    b = workload.batch()
    m = hgnn.Model(workload.num_layers, workload.hidden, 9, workload.edge_feat, 4,
                   workload.precision, workload.recompute, workload.delta)
    m.set_params(workload.params())
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    loss = torch.empty(1, device="cuda")

    def step():
        m.forward(db, pred, loss)
        m.backward()
        m.adam_step(lr=1e-3)

    m.forward(db, pred, loss, validate=True)
    step()
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            step()
    for _ in range(warmup):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    m.close()
    return {"graphs_per_s": b.num_graphs * steps / dt, "ms_per_step": 1e3 * dt / steps}


def multitask_rate(workload, steps, warmup, Tg=2, Tn=2):
    """Training step of the same GC stack with Tg graph-level and Tn node-level
    heads and a weighted loss (seeded synthetic targets)."""
    import numpy as np
    import torch
    from paper_2207_11333_amd import hgnn, synth
    b = workload.batch()
    rng = np.random.default_rng(workload.data_seed + 77)
    H = workload.hidden
    layers = workload.params()[:-(H * H + 2 * H + 1)]
    lim = np.sqrt(6.0 / (2 * H))
    heads = []
    for _ in range(Tg + Tn):
        heads += [rng.uniform(-lim, lim, H * H), rng.uniform(-0.1, 0.1, H),
                  rng.uniform(-lim, lim, H), rng.uniform(-0.1, 0.1, 1)]
    params = np.concatenate([layers] + heads).astype(np.float32)
    y = rng.normal(5.0, 1.5, size=(b.num_graphs, Tg)).astype(np.float32)
    yn = torch.tensor(rng.normal(0.0, 1.0, size=(b.num_nodes, Tn)).astype(np.float32),
                      device="cuda")
    m = hgnn.Model(workload.num_layers, H, 9, workload.edge_feat, 4, workload.precision,
                   workload.recompute, workload.delta, graph_heads=Tg, node_heads=Tn,
                   graph_weights=[1.0] + [0.5] * (Tg - 1), node_weights=[0.25] * Tn)
    m.set_params(params)
    db = hgnn.DeviceBatch.from_host(synth.Batch(b.graph_ptr, b.x, b.edge_index, b.edge_attr, y))
    pred = torch.empty(b.num_graphs, Tg, device="cuda")
    pn = torch.empty(b.num_nodes, Tn, device="cuda")
    loss = torch.empty(1, device="cuda")

    def step():
        m.forward(db, pred, loss, y_node=yn, pred_node=pn)
        m.backward()
        m.adam_step(lr=1e-3)

    m.forward(db, pred, loss, validate=True, y_node=yn, pred_node=pn)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    m.close()
    return {"graph_heads": Tg, "node_heads": Tn, "graphs_per_s": b.num_graphs * steps / dt,
            "ms_per_step": 1e3 * dt / steps}


def sage_gemm_flops(workload, N):
    """FLOPs of one GraphSAGE layer GEMM ([h || M] W^T), averaged over the
    layers (layer 0 reads the padded 16-wide input)."""
    H, L = workload.hidden, workload.num_layers
    ks = [2 * 16] + [2 * H] * (L - 1)
    return sum(2.0 * N * k * H for k in ks) / L


def cgcnn_aggregate_bytes(N, E, H, Fe):
    """Algorithmic bytes of one CGCNN gated aggregation: own gate halves
    (N x 2H) and gathered source halves (E x 2H), the layer input and output
    (N x H each), CSR arrays and edge attributes; FP32."""
    return 4 * (2 * H * N + 2 * H * E + 2 * H * N + (N + 1) + E + E * Fe)


def gc_rate(kind, workload, steps, warmup, precision=0, site=None):
    """Training step (CSR build, forward, backward, AdamW) of a GraphSAGE or
    CGCNN model of the workload's depth and width on the same batch; with a
    timer site, a second pass times that site's launches."""
    import torch
    from paper_2207_11333_amd import hgnn, synth
    b = workload.batch()
    m = hgnn.Model(workload.num_layers, workload.hidden, 9, workload.edge_feat, 4, precision,
                   0, 1.0, kind=kind)
    m.set_params(synth.init_gc_params(kind, workload.num_layers, workload.hidden, 2100))
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    loss = torch.empty(1, device="cuda")

    def step():
        m.forward(db, pred, loss)
        m.backward()
        m.adam_step(lr=1e-3)

    m.forward(db, pred, loss, validate=True)
    for _ in range(warmup):
        step()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        step()
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    out = {"graphs_per_s": b.num_graphs * steps / dt, "ms_per_step": 1e3 * dt / steps,
           "N": b.num_nodes, "E": b.num_edges}
    if site:
        m.timer_start(site, steps * workload.num_layers + 16)
        torch.cuda.synchronize()
        for _ in range(steps):
            step()
        torch.cuda.synchronize()
        out["site_ms_total"], out["site_launches"] = m.timer_read()
    m.close()
    return out


def gc_measure(workload, steps, warmup):
    out = {"workload": (f"{workload.num_layers} layers, hidden {workload.hidden}, "
                        f"{workload.num_graphs} molecules of {workload.n_lo}-{workload.n_hi} "
                        "atoms (the FP32 headline batch)")}
    for kind, site in (("sage", "update_gemm"), ("cgcnn", "aggregate")):
        r32 = gc_rate(kind, workload, steps, warmup, 0, site)
        r16 = gc_rate(kind, workload, steps, warmup, 1)
        out[kind] = {"fp32_graphs_per_s": r32["graphs_per_s"], "fp32_ms_per_step": r32["ms_per_step"],
                     "bf16_graphs_per_s": r16["graphs_per_s"], "bf16_ms_per_step": r16["ms_per_step"]}
        avg = r32["site_ms_total"] / 1e3 / max(1, r32["site_launches"])
        if kind == "sage":
            fl = sage_gemm_flops(workload, r32["N"])
            ach = fl / avg / 1e12
            out[kind]["roofline"] = {"kernel": "GraphSAGE layer GEMM, FP32", "bound": "mfma",
                                     "achieved": ach, "peak": FP32_PEAK_TFLOPS,
                                     "unit": "TFLOP/s", "frac": ach / FP32_PEAK_TFLOPS,
                                     "avg_us": avg * 1e6, "flops_per_launch": fl}
        else:
            nb = cgcnn_aggregate_bytes(r32["N"], r32["E"], workload.hidden, workload.edge_feat)
            ach = nb / avg / 1e9
            out[kind]["roofline"] = {"kernel": "CGCNN gated aggregation, FP32", "bound": "hbm",
                                     "achieved": ach, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                                     "frac": ach / HBM_PEAK_GBS, "avg_us": avg * 1e6,
                                     "bytes_per_launch": nb,
                                     "note": "cache-resident at this size"}
    return out


def serve_bench(qps=500.0, warm_s=2.0, measure_s=20.0, pool=48):
    """Open-loop Poisson arrivals at a fixed rate; latency is measured from the
    scheduled arrival time to the poll that observes completion."""
    import numpy as np
    from paper_2207_11333_amd import hgnn, synth
    sw = synth.SERVE_WORKLOAD
    shape = synth.ModelShape(sw["num_layers"], sw["hidden"], 9, sw["edge_feat"])
    m = hgnn.Model(sw["num_layers"], sw["hidden"], 9, sw["edge_feat"], 4, sw["precision"], 0,
                   sw["delta"])
    m.set_params(synth.init_params(shape, sw["weight_seed"]))
    rng = np.random.default_rng(sw["request_seed"])
    reqs = [synth.make_request(rng, sw["mol_lo"], sw["mol_hi"], sw["n_lo"], sw["n_hi"],
                               sw["edge_feat"]) for _ in range(pool)]
    m.serve_start(hbm_budget_bytes=16 << 30, max_batch_nodes=32768, max_batch_edges=73728,
                  max_batch_graphs=1024, num_lanes=4, queue_capacity=65536, use_graphs=1)
    arr = np.random.default_rng(sw["arrival_seed"])
    total = warm_s + measure_s
    times = np.cumsum(arr.exponential(1.0 / qps, size=int(qps * total * 1.2) + 16))
    times = times[times < total]
    pending = {}
    lat, graphs_done = [], 0
    t0 = time.perf_counter()
    i = 0
    while i < len(times) or pending:
        now = time.perf_counter() - t0
        while i < len(times) and times[i] <= now:
            r = reqs[i % pool]
            t = m.serve_submit(r)
            if t >= 0:
                pending[t] = (times[i], r.num_graphs)
            i += 1
        done = []
        for t, (ts, nb) in pending.items():
            if m.serve_poll(t, nb) is not None:
                fin = time.perf_counter() - t0
                if ts >= warm_s:
                    lat.append(fin - ts)
                    graphs_done += nb
                done.append(t)
        for t in done:
            del pending[t]
        if now > total + 30:
            break
    stats = m.serve_stats()
    sat = serve_saturation(m, reqs)
    m.serve_stop()
    m.close()
    lat = np.sort(np.asarray(lat)) * 1e3
    return {"workload": "serving: 6-layer PNA, hidden 128, BF16; requests of 1-256 molecules "
                        "of 5-70 atoms (pool of %d synthetic requests), Poisson arrivals" % pool,
            "qps": qps, "window_s": measure_s, "requests_measured": int(lat.size),
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None,
            "graphs_per_s": graphs_done / measure_s, "batches": stats["batches"],
            "graph_replays": stats["graph_replays"], "saturation": sat}


def serve_saturation(m, reqs, inflight=64, warm_s=1.0, measure_s=5.0):
    """Closed loop: keep `inflight` requests submitted at all times; the
    completion rate is the server's capacity at this request mix."""
    import numpy as np
    pending, lat, graphs_done, reqs_done = {}, [], 0, 0
    t0 = time.perf_counter()
    i = 0
    while True:
        now = time.perf_counter() - t0
        if now > warm_s + measure_s:
            break
        while len(pending) < inflight:
            r = reqs[i % len(reqs)]
            t = m.serve_submit(r)
            if t < 0:
                break
            pending[t] = (time.perf_counter() - t0, r.num_graphs)
            i += 1
        done = []
        for t, (ts, nb) in pending.items():
            if m.serve_poll(t, nb) is not None:
                fin = time.perf_counter() - t0
                if ts >= warm_s:
                    lat.append(fin - ts)
                    graphs_done += nb
                    reqs_done += 1
                done.append(t)
        for t in done:
            del pending[t]
    t_drain = time.perf_counter()
    while pending and time.perf_counter() - t_drain < 30.0:  # drain
        for t, (ts, nb) in list(pending.items()):
            if m.serve_poll(t, nb) is not None:
                del pending[t]
    if pending:
        raise RuntimeError(f"{len(pending)} serving requests did not complete")
    lat = np.sort(np.asarray(lat)) * 1e3
    return {"inflight": inflight, "graphs_per_s": graphs_done / measure_s,
            "requests_per_s": reqs_done / measure_s,
            "p50_ms": float(np.percentile(lat, 50)) if lat.size else None,
            "p99_ms": float(np.percentile(lat, 99)) if lat.size else None}


def loader_bench(steps=100, warmup=10, nbatches=16):
    """Training fed from the packed graph store on local disk (reader threads
    into pinned buffers, copy overlapped with compute) against the same
    batches already resident in HBM; plus the reader alone."""
    import tempfile
    import torch
    from paper_2207_11333_amd import graphstore, hgnn, synth
    w = synth.WORKLOADS["c1_train_fp32"]
    batches = [synth.make_batch(w.data_seed + 1000 + i, w.num_graphs, w.n_lo, w.n_hi,
                                w.edge_feat) for i in range(nbatches)]
    fd, path = tempfile.mkstemp(suffix=".hgnnstore")
    os.close(fd)
    try:
        entries = graphstore.write_store(path, batches, edge_feat=w.edge_feat)
        m = hgnn.Model(w.num_layers, w.hidden, 9, w.edge_feat, 4, w.precision, w.recompute,
                       w.delta)
        m.set_params(w.params())
        pred = torch.empty(w.num_graphs, device="cuda")
        loss = torch.empty(1, device="cuda")

        def run(get):
            for i in range(warmup):
                m.forward(get(i), pred, loss)
                m.backward()
                m.adam_step()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            for i in range(steps):
                m.forward(get(warmup + i), pred, loss)
                m.backward()
                m.adam_step()
            torch.cuda.synchronize()
            return w.num_graphs * steps / (time.perf_counter() - t0)

        dbs = [hgnn.DeviceBatch.from_host(b) for b in batches]
        resident = run(lambda i: dbs[i % nbatches])
        store = hgnn.GraphStore(path, io_threads=4, host_slots=4)
        streamed = run(lambda i: store.next())
        # the reader alone: records per second through pinned memory to HBM
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        nread = 4 * nbatches
        for _ in range(nread):
            store.next()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        store.close()
        m.close()
        rec = sum(e["bytes"] for e in entries) / nbatches
        return {"workload": f"c1 shapes, {nbatches} distinct batches in one store file",
                "resident_graphs_per_s": resident, "store_graphs_per_s": streamed,
                "store_vs_resident": streamed / resident,
                "reader_batches_per_s": nread / dt, "reader_MB_per_s": nread * rec / dt / 1e6,
                "record_bytes": rec}
    finally:
        os.unlink(path)


def aggregate_bytes(N, E, H, Fe):
    """Algorithmic bytes of one forward aggregation launch (S2): gathered Q
    rows (E x H), own P rows (N x H), CSR arrays and edge attributes read; the
    aggregates A (N x 4H, FP32) and the arg bytes (N x 2H) written."""
    return 4 * H * E + 4 * H * N + 4 * (N + 1) + 4 * E + 4 * E * Fe + 16 * H * N + 2 * H * N


def aggregate_bwd_bytes(N, E, H, Fe, fused=False):
    """Algorithmic bytes of one aggregation-adjoint launch (S7): dA (4H), mean
    and std (2H), arg bytes (2H) and P (H) per node, gathered Q (H) per edge and
    the CSR read; per-edge dm (E x H), D_in (N x H) and De (N x H Fe) written.
    Fused with the aggregate-input gradient, du (H per node) is read instead
    of dA (the weights, a few MB, are left out)."""
    reads = (4 if fused else 16) * H * N + 8 * H * N + 2 * H * N + 4 * H * N + 4 * H * E
    reads += 4 * (N + 1) + 4 * E + 4 * E * Fe
    writes = 4 * H * E + 4 * H * N + 4 * H * N * Fe
    return reads + writes


def c3_measure(steps=8, warmup=2):
    """One GPU's share of the large data-parallel step: 8 layers, hidden 256,
    1024 molecules, BF16 linears, recomputation on.  Times the step, every
    launch site (the two aggregation kernels against the HBM roofline), the
    phases, and the device memory with recomputation on and off."""
    from paper_2207_11333_amd import synth
    w = synth.WORKLOADS["c3_large_bf16"]
    r = train_rate(w, steps, warmup, sites=True, phases=True)
    out = {"graphs_per_s": r["graphs_per_s"], "ms_per_step": r["ms_per_step"],
           "nodes": r["N"], "edges": r["E"]}
    for site in ("aggregate", "aggregate_bwd"):
        st = r["sites"][site]
        out[site] = {"avg_us": st["avg_us"], "bytes_per_launch": st["bytes_per_launch"],
                     "achieved": st["achieved"], "unit": "GB/s", "peak": HBM_PEAK_GBS,
                     "frac": st["frac"], "launches": st["launches"],
                     "traffic": measured_traffic(*AGGREGATE_TRAFFIC[site])}
    out["workload"] = ("c3_large_bf16: 8-layer PNA, hidden 256, 1024 molecules of 10-70 atoms, "
                       "BF16 linears, FP32 aggregation, recomputation on")
    out["sites"] = r["sites"]
    out["phases"] = r["phases"]
    # the same step with FP32 linears: the BF16 / FP32 ratio where the
    # linears dominate the step
    import dataclasses
    r32 = train_rate(dataclasses.replace(w, precision=0), 4, 1)
    out["fp32_graphs_per_s"] = r32["graphs_per_s"]
    out["bf16_ratio_vs_fp32"] = r["graphs_per_s"] / r32["graphs_per_s"]
    out["memory"] = {"recompute_on_bytes": step_memory(w, 1),
                     "recompute_off_bytes": step_memory(w, 0),
                     "note": "device memory taken by the context and one training step: the "
                             "drop in free device memory from before the model is created to "
                             "after its first step (parameters, moments, staged weights, "
                             "workspace, the batch)"}
    copy = copy_bandwidth()
    out["copy_gbs"] = copy
    for site in ("aggregate", "aggregate_bwd"):
        out[site]["frac_of_copy"] = out[site]["achieved"] / copy
    return out


def step_memory(w, recompute):
    """Free device memory before creating the model minus after one step."""
    import dataclasses
    import gc
    import torch
    from paper_2207_11333_amd import hgnn
    w = dataclasses.replace(w, recompute=recompute)
    b = w.batch()
    torch.cuda.synchronize()
    gc.collect()
    torch.cuda.empty_cache()
    free0 = torch.cuda.mem_get_info()[0]
    m = hgnn.Model(w.num_layers, w.hidden, 9, w.edge_feat, 4, w.precision, recompute, w.delta)
    m.set_params(w.params())
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    loss = torch.empty(1, device="cuda")
    m.forward(db, pred, loss)
    m.backward()
    m.adam_step(lr=1e-3)
    torch.cuda.synchronize()
    used = free0 - torch.cuda.mem_get_info()[0]
    m.close()
    del db, pred, loss
    return int(used)


def accuracy_sample(w, ngraphs=32):
    """Prediction and loss of the first `ngraphs` graphs of the workload's
    batch on the GPU against the FP64 oracle: L2 ratio and max|a-r|/max|r|."""
    import numpy as np
    import torch
    import oracle
    from paper_2207_11333_amd import hgnn, synth
    b = synth.select_graphs(w.batch(), range(ngraphs))
    params = w.params()
    m = hgnn.Model(w.num_layers, w.hidden, 9, w.edge_feat, 4, w.precision, w.recompute,
                   w.delta)
    m.set_params(params)
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    loss = torch.empty(1, device="cuda")
    m.forward(db, pred, loss, validate=True)
    torch.cuda.synchronize()
    a = pred.cpu().numpy().astype(np.float64)
    m.close()
    # one BLAS thread: a pool of spinning BLAS threads would take host cores
    # from the launching thread of the GPU timings that follow
    try:
        import threadpoolctl
        with threadpoolctl.threadpool_limits(limits=1):
            rec = oracle.forward(params.astype(np.float64), b, w.num_layers, w.hidden, w.delta)
    except ImportError:
        rec = oracle.forward(params.astype(np.float64), b, w.num_layers, w.hidden, w.delta)
    r = np.asarray(rec.y, np.float64)
    return {"graphs": ngraphs, "atoms": b.num_nodes,
            "pred_rel_l2": float(np.linalg.norm(a - r) / np.linalg.norm(r)),
            "pred_rel_max": float(np.abs(a - r).max() / np.abs(r).max()),
            "loss_rel": float(abs(loss.item() - rec.loss) / abs(rec.loss))}


def copy_bandwidth(mib=1024, reps=20):
    """Practical HBM bandwidth: a plain float4 copy of `mib` MiB (read + write)."""
    import torch
    from paper_2207_11333_amd import hgnn
    n = mib << 18
    src = torch.ones(n, device="cuda")
    dst = torch.empty_like(src)
    hgnn.calib_copy(src, dst)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        hgnn.calib_copy(src, dst)
    e1.record()
    torch.cuda.synchronize()
    sec = e0.elapsed_time(e1) / 1e3 / reps
    del src, dst
    return 2 * n * 4 / sec / 1e9


def _oracle_steps(workload, ngraphs, budget_s):
    """FP64 oracle train steps (forward, backward, AdamW) on the first
    `ngraphs` graphs of the workload's batch for about budget_s seconds."""
    import numpy as np
    import oracle
    from paper_2207_11333_amd import synth
    sample = synth.select_graphs(workload.batch(), range(ngraphs))
    params = workload.params().astype(np.float64)
    m = np.zeros_like(params)
    v = np.zeros_like(params)
    n_graphs, t = 0, 0
    t0 = time.perf_counter()
    while time.perf_counter() - t0 < budget_s:
        rec = oracle.forward(params, sample, workload.num_layers, workload.hidden, workload.delta)
        g, _, _ = oracle.backward(rec)
        t += 1
        params, m, v = oracle.adamw(params, g, m, v, t)
        n_graphs += sample.num_graphs
    dt = time.perf_counter() - t0
    return n_graphs / dt, t, sample.num_nodes, dt


def _cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return None


def cpu_baseline(workload, budget_s=7.0):
    """The FP64 oracle on the host: the headline workload's first 16 graphs with
    every BLAS thread (the reported value) and pinned to one thread, and the
    small workload's first 16 graphs."""
    from paper_2207_11333_amd import synth
    try:
        import threadpoolctl
    except ImportError:
        threadpoolctl = None
    threads = None
    if threadpoolctl is not None:
        info = threadpoolctl.threadpool_info()
        threads = max([i.get("num_threads", 1) for i in info] + [1])
    v_all, t_all, atoms, dt_all = _oracle_steps(workload, 16, budget_s)
    if threadpoolctl is not None:
        with threadpoolctl.threadpool_limits(limits=1):
            v_one, t_one, _, dt_one = _oracle_steps(workload, 16, budget_s * 0.7)
    else:
        v_one = t_one = dt_one = None
    w0 = synth.WORKLOADS["c0_small_fp32"]
    v_c0, t_c0, atoms0, dt_c0 = _oracle_steps(w0, 16, budget_s * 0.5)
    return {"value": v_all, "unit": "graphs/s", "cores": threads or 1, "kind": "oracle",
            "sample": f"{t_all} FP64 oracle train steps (forward + backward + AdamW) on the "
                      f"first 16 graphs ({atoms} atoms) of the same batch, {dt_all:.1f} s, "
                      "all BLAS threads",
            "one_thread": {"value": v_one, "steps": t_one, "seconds": dt_one},
            "c0_small": {"value": v_c0, "steps": t_c0, "atoms": atoms0, "seconds": dt_c0},
            "blas_threads": threads, "host_cores": len(os.sched_getaffinity(0)),
            "cpu_model": _cpu_model()}


def main():
    ap = argparse.ArgumentParser(description=__doc__)
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=100)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--qps", type=float, default=500.0, help="serving request rate")
    ap.add_argument("--calib-copy", action="store_true",
                    help="first run a 256 MiB copy kernel (counter calibration)")
    ap.add_argument("--no-extras", action="store_true",
                    help="skip the BF16 and serving measurements")
    ap.add_argument("--workload", default="c1_train_fp32",
                    choices=["c1_train_fp32", "c2_train_bf16"],
                    help="training workload of the headline line (the BF16 choice is "
                         "for profiling; the default line is the FP32 one)")
    ap.add_argument("--only-large", action="store_true",
                    help="run only the large-configuration measurement (for profiling) "
                         "and print its JSON")
    ap.add_argument("--only-gc", choices=["sage", "cgcnn"], default=None,
                    help="run only the training step of that layer kind on the headline "
                         "batch (for profiling) and print its JSON")
    args = ap.parse_args()
    world = int(os.environ.get("WORLD_SIZE", "1"))
    if args.gpus != 1 or world != 1:
        print(json.dumps({"error": "hgnn runs on one GPU: the data-parallel gradient "
                          "all-reduce across GPUs is not implemented; run with --gpus 1"}))
        sys.exit(2)

    import torch
    from paper_2207_11333_amd import synth
    torch.cuda.set_device(0)
    w = synth.WORKLOADS[args.workload]
    bf16 = w.precision == 1
    if args.calib_copy:
        from paper_2207_11333_amd import hgnn
        src = torch.ones(64 << 20, device="cuda")
        dst = torch.empty_like(src)
        hgnn.calib_copy(src, dst)
        torch.cuda.synchronize()
        del src, dst
    if args.only_gc:
        _log(f"bench: {args.only_gc} only")
        print(json.dumps({args.only_gc: gc_rate(args.only_gc, w, args.steps, args.warmup,
                                                w.precision)}), flush=True)
        return
    if args.only_large:
        _log("bench: large configuration only")
        print(json.dumps({"c3": c3_measure()}), flush=True)
        return
    _log(f"bench: {w.name} steps={args.steps} warmup={args.warmup}")
    r = train_rate(w, args.steps, args.warmup, sites=True, phases=True)
    _log(f"bench: {'bf16' if bf16 else 'fp32'} {r['graphs_per_s']:.1f} graphs/s, "
         f"{r['ms_per_step']:.3f} ms/step")
    roof = dominant_roofline(r["sites"])
    _log(f"bench: dominant site {roof['site']} {roof['us_per_step']:.1f} us/step, "
         f"{roof['achieved']:.1f} {roof['unit']} ({100 * roof['frac']:.1f}% of peak)")
    wdesc = (f"{w.name}: {w.num_layers}-layer PNA GCNN, hidden {w.hidden}, {w.num_graphs} "
             f"synthetic molecules of {w.n_lo}-{w.n_hi} atoms, {w.edge_feat} edge feature, "
             f"{'BF16 linears, FP32 aggregation' if bf16 else 'FP32'}, "
             "CSR build + forward + backward + Adam per step")
    line = {
        "metric": "train graphs/s fwd+bwd (BF16 vs FP32) at stated error; serve p50/p99 ms",
        "value": r["graphs_per_s"], "unit": "graphs/s", "n_gpus": 1, "steps": args.steps,
        "warmup": args.warmup, "ms_per_step": r["ms_per_step"], "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "bf16" if bf16 else "f32",
        "data": "synthetic",
        "config": {"workload": wdesc,
                   "graphs_per_step": r["B"], "nodes": r["N"], "edges": r["E"],
                   "layers": w.num_layers, "hidden": w.hidden,
                   "precision": "bf16" if bf16 else "fp32"},
        "roofline": roof,
        "sites": r["sites"],
        "phases": r["phases"],
    }
    if not args.no_extras and not bf16:
        rg = train_rate_graph(w, args.steps, args.warmup)
        _log(f"bench: fp32 graph-replayed {rg['graphs_per_s']:.1f} graphs/s")
        line["fp32_graph_replay"] = {"value": rg["graphs_per_s"], "unit": "graphs/s",
                                     "ms_per_step": rg["ms_per_step"]}
        wb = synth.WORKLOADS["c2_train_bf16"]
        rb = train_rate(wb, args.steps, args.warmup, sites=True, phases=True)
        rbg = train_rate_graph(wb, args.steps, args.warmup)
        _log(f"bench: bf16 {rb['graphs_per_s']:.1f} graphs/s, graph-replayed "
             f"{rbg['graphs_per_s']:.1f}")
        line["bf16"] = {"workload": wb.name, "value": rb["graphs_per_s"], "unit": "graphs/s",
                        "ms_per_step": rb["ms_per_step"], "sites": rb["sites"],
                        "phases": rb["phases"],
                        "ratio_vs_fp32": rb["graphs_per_s"] / r["graphs_per_s"],
                        "graph_replay_value": rbg["graphs_per_s"],
                        "graph_replay_ratio_vs_fp32": rbg["graphs_per_s"] / rg["graphs_per_s"]}
        mt = multitask_rate(w, args.steps, args.warmup)
        mt["ratio_vs_single_head"] = mt["graphs_per_s"] / r["graphs_per_s"]
        line["multitask"] = mt
        _log(f"bench: multitask ({mt['graph_heads']} graph + {mt['node_heads']} node heads) "
             f"{mt['graphs_per_s']:.1f} graphs/s")
        _log("bench: GraphSAGE and CGCNN layer kinds")
        line["gc_layers"] = gc_measure(w, args.steps, args.warmup)
        _log("bench: " + ", ".join(
            f"{k} {line['gc_layers'][k]['fp32_graphs_per_s']:.0f} (bf16 "
            f"{line['gc_layers'][k]['bf16_graphs_per_s']:.0f})" for k in ("sage", "cgcnn"))
            + " graphs/s")
        _log("bench: large configuration")
        line["c3"] = c3_measure()
        _log(f"bench: c3 {line['c3']['graphs_per_s']:.1f} graphs/s; aggregation "
             f"{line['c3']['aggregate']['achieved']:.0f} GB/s, adjoint "
             f"{line['c3']['aggregate_bwd']['achieved']:.0f} GB/s")
        _log("bench: serving")
        line["serve"] = serve_bench(qps=args.qps)
        _log(f"bench: serve p50 {line['serve']['p50_ms']} ms p99 {line['serve']['p99_ms']} ms; "
             f"capacity {line['serve']['saturation']['graphs_per_s']:.0f} molecules/s")
        _log("bench: training fed from the packed graph store")
        line["loader"] = loader_bench()
        _log(f"bench: store {line['loader']['store_graphs_per_s']:.1f} graphs/s vs resident "
             f"{line['loader']['resident_graphs_per_s']:.1f}; reader "
             f"{line['loader']['reader_MB_per_s']:.0f} MB/s")
    if not args.no_extras:
        # after every GPU timing: the oracle runs on the host
        _log("bench: prediction and loss against the FP64 oracle")
        line["error_vs_fp64"] = {w.name: accuracy_sample(w)}
        if not bf16:
            wb = synth.WORKLOADS["c2_train_bf16"]
            line["error_vs_fp64"][wb.name] = accuracy_sample(wb)
    if not args.no_cpu_baseline:
        _log("bench: timing the FP64 oracle on the host")
        line["cpu_baseline"] = cpu_baseline(w)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
