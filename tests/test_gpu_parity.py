"""Parity of the HIP path (through the C-ABI) with the FP64 oracle.

Tolerances: FP32 path 1e-5 relative (L2 norm ratio per tensor) on outputs,
loss and every parameter-gradient tensor; BF16 path 2e-2 relative on the
outputs and the loss, gradient error reported.  Integer CSR work is bit-exact.
Gradient comparisons use decision replay: the oracle adopts the GPU's min/max
and ReLU decisions only where its own FP64 values are within a tie window.
"""
import math
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

import oracle
from paper_2207_11333_amd import synth

pytestmark = pytest.mark.gpu

TAU_FP32 = 1e-4
TAU_BF16 = 3e-2


def _hgnn():
    from paper_2207_11333_amd import hgnn
    return hgnn


def rel(a, r):
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    nr = np.linalg.norm(r)
    return float(np.linalg.norm(a - r) / (nr if nr > 0 else 1.0))


def maxrel(a, r):
    """Element-wise error on the scale of the reference: max|a - r| / max|r|."""
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    mr = np.abs(r).max() if r.size else 0.0
    return float(np.abs(a - r).max() / (mr if mr > 0 else 1.0)) if r.size else 0.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def make_model(L, H, Fe, prec=0, recompute=0, delta=1.0, maxd=4, F0=9):
    return _hgnn().Model(L, H, F0, Fe, maxd, prec, recompute, delta)


def run_train_step(model, batch, params, backward=True):
    hg = _hgnn()
    model.set_params(params)
    db = hg.DeviceBatch.from_host(batch)
    B = batch.num_graphs
    pred = torch.empty(B, device="cuda")
    loss = torch.empty(1, device="cuda")
    model.forward(db, pred, loss, validate=True)
    out = {"db": db, "pred": pred, "loss": loss}
    if backward:
        model.backward()
        out["grads"] = model.grads()
    torch.cuda.synchronize()
    return out


def gpu_decisions(model, L, H, N, B):
    am, ax, rl = [], [], []
    for l in range(L):
        a = model.fetch(8, l, (N, 2 * H), torch.uint8).cpu().numpy().astype(np.int64)
        am.append(a[:, :H])
        ax.append(a[:, H:])
        rl.append(model.fetch(11, l, (N, H), torch.float32).cpu().numpy() > 0)
    q = model.fetch(9, 0, (B, H), torch.float32).cpu().numpy()
    return oracle.Decisions(am, ax, rl, q > 0)


def grad_report(model, g_gpu, g_ref, shape, elementwise=False):
    """Per parameter tensor: the L2 ratio, or (elementwise) max|a-r|/max|r|."""
    offs = shape.offsets()
    out = {}
    f = maxrel if elementwise else rel
    for name, (off, shp) in offs.items():
        n = int(np.prod(shp))
        out[name] = f(g_gpu[off:off + n], g_ref[off:off + n])
    return out


# element-wise gate of the FP32 path, beside the 1e-5 L2 gate
ELEM_FP32 = 1e-4


# ---------------------------------------------------------------------------
# S0: CSR, bit-exact
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name,permute", [("c0_small_fp32", False), ("c1_train_fp32", False),
                                          ("c1_train_fp32", True)])
def test_csr_bit_exact(name, permute):
    w = synth.WORKLOADS[name]
    b = w.batch()
    if permute:
        p = np.random.default_rng(5).permutation(b.num_edges)
        b = synth.Batch(b.graph_ptr, b.x, b.edge_index[:, p].copy(),
                        None if b.edge_attr is None else b.edge_attr[p].copy(), b.y)
    say(f"csr {name} permute={permute} N={b.num_nodes} E={b.num_edges}")
    m = make_model(1, 16, w.edge_feat)
    m.prepare(_hgnn().DeviceBatch.from_host(b), validate=True)
    ref = oracle.csr_build(b.graph_ptr, b.edge_index, b.num_nodes)
    N, E = b.num_nodes, b.num_edges
    got = {k: m.fetch(i, 0, (n,)).cpu().numpy() for k, i, n in
           [("rowptr", 0, N + 1), ("csr_src", 1, E), ("csr_eid", 2, E), ("deg", 3, N),
            ("srcptr", 4, N + 1), ("t2csr", 5, E), ("node_graph", 6, N)]}
    for k, v in got.items():
        assert np.array_equal(v, getattr(ref, k)), k
    m.close()


# ---------------------------------------------------------------------------
# the hand-worked path graph, embedded in a 16-wide model
# ---------------------------------------------------------------------------

def _path3_embedded(x):
    H, F = 16, 1
    shape = synth.ModelShape(1, H, F, 0)
    offs = shape.offsets()
    p = np.zeros(shape.num_params(), np.float32)
    o, _ = offs["l0.Wm"]
    p[o + 0 * (2 * F) + 1] = 1.0                      # row 0: [h_dst, h_src] = [0, 1]
    o, _ = offs["l0.Wp"]
    ld = F + 12 * H
    p[o + 0] = 1.0                                    # self
    for j in range(3):
        for a in range(4):
            p[o + F + j * 4 * H + a * H + 0] = 1.0    # feature 0 of every block
    o, _ = offs["W1"]
    p[o] = 1.0
    o, _ = offs["w2"]
    p[o] = 1.0
    b = synth.Batch(np.array([0, 3], np.int32), np.array(x, np.float32)[:, None],
                    np.array([[0, 1, 1, 2], [1, 0, 2, 1]], np.int32), None,
                    np.zeros(1, np.float32))
    return b, p, shape


@pytest.mark.parametrize("x,y,loss,dx", [
    ([1, 2, 4], 23.987338224741155, 575.3923951081281,
     [67.41874608958747, 303.83961751338796, 118.84576193948516]),
    ([1, 2, 1], 16.558939991024037, 274.1984936263351,
     [99.79223808806668, 209.74657321963778, 28.789882279492826])])
def test_hand_worked_example_on_gpu(x, y, loss, dx):
    hg = _hgnn()
    b, p, shape = _path3_embedded(x)
    m = hg.Model(1, 16, 1, 0, 4, 0, 0, math.log(2.0))
    out = run_train_step(m, b, p)
    assert out["pred"].item() == pytest.approx(y, rel=1e-5)
    assert out["loss"].item() == pytest.approx(loss, rel=1e-5)
    net = hg.PNANet(m, p)
    db = hg.DeviceBatch.from_host(b)
    xt = db.x.clone().requires_grad_(True)
    pred = net(db, xt)
    ((pred - db.y) ** 2).mean().backward()
    np.testing.assert_allclose(xt.grad.cpu().numpy()[:, 0], dx, rtol=1e-5)
    m.close()


# ---------------------------------------------------------------------------
# FP32 forward and backward parity
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("name", ["c0_small_fp32", "c1_train_fp32"])
def test_fp32_forward_backward_parity(name):
    w = synth.WORKLOADS[name]
    b, params = w.batch(), w.params()
    L, H = w.num_layers, w.hidden
    say(f"fp32 parity {name}: N={b.num_nodes} E={b.num_edges}")
    m = make_model(L, H, w.edge_feat, 0, 0, w.delta)
    out = run_train_step(m, b, params)
    rec = oracle.forward(params, b, L, H, w.delta)
    pred = out["pred"].cpu().numpy()
    r_pred, e_pred = rel(pred, rec.y), maxrel(pred, rec.y)
    r_loss = rel([out["loss"].item()], [rec.loss])
    say(f"  pred rel {r_pred:.2e} (element-wise {e_pred:.2e})  loss rel {r_loss:.2e}")
    for l in range(L):
        A = m.fetch(7, l, (b.num_nodes, 4 * H), torch.float32).cpu().numpy()
        hl = m.fetch(11, l, (b.num_nodes, H), torch.float32).cpu().numpy()
        say(f"  layer {l}: A rel {rel(A, rec.layers[l].A):.2e} (element-wise "
            f"{maxrel(A, rec.layers[l].A):.2e})  h rel {rel(hl, rec.layers[l].h_out):.2e} "
            f"(element-wise {maxrel(hl, rec.layers[l].h_out):.2e})")
        assert rel(A, rec.layers[l].A) <= 1e-5
        assert rel(hl, rec.layers[l].h_out) <= 1e-5
        assert maxrel(A, rec.layers[l].A) <= ELEM_FP32
        assert maxrel(hl, rec.layers[l].h_out) <= ELEM_FP32
    assert r_pred <= 1e-5 and r_loss <= 1e-5 and e_pred <= ELEM_FP32
    dec = gpu_decisions(m, L, H, b.num_nodes, b.num_graphs)
    g_ref, _, stats = oracle.backward(rec, hint=dec, tau=TAU_FP32)
    g = out["grads"].cpu().numpy()
    rep = grad_report(m, g, g_ref, w.shape)
    erep = grad_report(m, g, g_ref, w.shape, elementwise=True)
    worst = max(rep, key=rep.get)
    eworst = max(erep, key=erep.get)
    say(f"  adopted decisions {stats}; worst grad {worst} rel {rep[worst]:.2e}; "
        f"worst element-wise {eworst} {erep[eworst]:.2e}")
    for k, v in rep.items():
        assert v <= 1e-5, (k, v)
    for k, v in erep.items():
        assert v <= ELEM_FP32, (k, v)
    m.close()


@pytest.mark.parametrize("Fe", [1, 2])
def test_large_batch_fp32_parity(Fe):
    """A batch above 16,384 atoms, where the message weight gradient takes the
    De rows apart (their column sums in a GEMM of their own), and of at least
    512 graphs, where the head weight gradients are summed in graph chunks:
    FP32 parity of predictions, loss and every gradient tensor (decision
    replay), with a 2-layer hidden-32 model so that the FP64 oracle stays
    quick."""
    b = synth.make_batch(777 + Fe, 520, 20, 50, Fe)
    assert b.num_nodes >= 16384 and b.num_graphs >= 512
    L, H, delta = 2, 32, 1.3
    shape = synth.ModelShape(L, H, 9, Fe)
    params = synth.init_params(shape, 99 + Fe)
    say(f"large fp32 Fe={Fe}: N={b.num_nodes} E={b.num_edges}")
    m = make_model(L, H, Fe, 0, 0, delta)
    out = run_train_step(m, b, params)
    rec = oracle.forward(params, b, L, H, delta)
    pred = out["pred"].cpu().numpy()
    r_pred, e_pred = rel(pred, rec.y), maxrel(pred, rec.y)
    r_loss = rel([out["loss"].item()], [rec.loss])
    dec = gpu_decisions(m, L, H, b.num_nodes, b.num_graphs)
    g_ref, _, stats = oracle.backward(rec, hint=dec, tau=TAU_FP32)
    g = out["grads"].cpu().numpy()
    rep = grad_report(m, g, g_ref, shape)
    erep = grad_report(m, g, g_ref, shape, elementwise=True)
    worst = max(rep, key=rep.get)
    eworst = max(erep, key=erep.get)
    say(f"  pred rel {r_pred:.2e} (element-wise {e_pred:.2e}) loss rel {r_loss:.2e}; "
        f"worst grad {worst} {rep[worst]:.2e}; element-wise {eworst} {erep[eworst]:.2e}; "
        f"adopted {stats}")
    assert r_pred <= 1e-5 and r_loss <= 1e-5 and e_pred <= ELEM_FP32
    for k, v in rep.items():
        assert v <= 1e-5, (k, v)
    for k, v in erep.items():
        assert v <= ELEM_FP32, (k, v)
    m.close()


def test_recompute_matches_stored_activations():
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    m0 = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    m1 = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 1, w.delta)
    o0 = run_train_step(m0, b, params)
    o1 = run_train_step(m1, b, params)
    assert torch.equal(o0["pred"], o1["pred"])
    assert torch.equal(o0["grads"], o1["grads"])
    m0.close()
    m1.close()


def test_determinism_bitwise():
    w = synth.WORKLOADS["c1_train_fp32"]
    b, params = w.batch(), w.params()
    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    o1 = run_train_step(m, b, params)
    g1, p1 = o1["grads"].clone(), o1["pred"].clone()
    s = torch.cuda.Stream()
    with torch.cuda.stream(s):
        o2 = run_train_step(m, b, params)
    torch.cuda.synchronize()
    assert torch.equal(p1, o2["pred"])
    assert torch.equal(g1, o2["grads"])
    m.close()


def test_autograd_functions_match_fused_entry_points():
    hg = _hgnn()
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    out = run_train_step(m, b, params)
    net = hg.PNANet(m, params)
    db = hg.DeviceBatch.from_host(b)
    pred = net(db)
    loss = ((pred - db.y) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    assert torch.equal(pred.detach(), out["pred"])
    g = net.packed_grad()
    assert rel(g.cpu().numpy(), out["grads"].cpu().numpy()) <= 1e-6
    m.close()


@pytest.mark.parametrize("name", ["c1_train_fp32", "c2_train_bf16"])
def test_deferred_joins_match_per_layer_joins(name):
    """The fused backward leaves each layer's weight-gradient stream to be
    joined at the next layer's aggregation adjoint; the per-operation layer
    entries (driven here by PNANet) join every layer at once.  At the full
    headline size, where the weight-gradient GEMMs run long beside the
    input-gradient chain, both give the same gradients (the loss gradient is
    formed by torch on one side and by the head kernel on the other, hence a
    tolerance instead of bitwise equality; in BF16 that difference can move a
    few operand roundings).  A missed wait would show as a far larger error."""
    hg = _hgnn()
    w = synth.WORKLOADS[name]
    b, params = w.batch(), w.params()
    say(f"deferred joins: {name} N={b.num_nodes} E={b.num_edges}")
    m = make_model(w.num_layers, w.hidden, w.edge_feat, w.precision, w.recompute, w.delta)
    out = run_train_step(m, b, params)
    net = hg.PNANet(m, params)
    db = hg.DeviceBatch.from_host(b)
    pred = net(db)
    loss = ((pred - db.y) ** 2).mean()
    loss.backward()
    torch.cuda.synchronize()
    assert torch.equal(pred.detach(), out["pred"])
    r = rel(net.packed_grad().cpu().numpy(), out["grads"].cpu().numpy())
    say(f"  gradient rel {r:.2e}")
    assert r <= (1e-5 if w.precision else 1e-6)
    m.close()


def test_gpu_path_central_differences():
    """FP32 finite differences through the GPU forward (loose: FP32 noise)."""
    hg = _hgnn()
    b = synth.make_batch(77, 4, 5, 12, 1)
    shape = synth.ModelShape(2, 16, 9, 1)
    params = synth.init_params(shape, 78).astype(np.float64)
    m = hg.Model(2, 16, 9, 1, 4, 0, 0, 1.0)
    out = run_train_step(m, b, params.astype(np.float32))
    g = out["grads"].cpu().numpy()
    db = hg.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    loss = torch.empty(1, device="cuda")
    idx = np.argsort(-np.abs(g))[:12]
    good = 0
    for j in idx:
        hstep = 1e-3 * max(1.0, abs(params[j]))
        vals = []
        for sgn in (1, -1):
            p = params.copy()
            p[j] += sgn * hstep
            m.set_params(p.astype(np.float32))
            m.forward(db, pred, loss)
            torch.cuda.synchronize()
            vals.append(loss.item())
        fd = (vals[0] - vals[1]) / (2 * hstep)
        ok = abs(fd - g[j]) <= 2e-2 * abs(g[j]) + 1e-3 * abs(g).max()
        say(f"  fd coord {j}: fd {fd:.6g} grad {g[j]:.6g} {'ok' if ok else 'off'}")
        good += ok
    # a step may cross a ReLU or min/max kink: allow two of twelve to miss
    assert good >= 10
    m.close()


def test_adamw_step_isolated():
    """The GPU AdamW given the GPU gradient equals the oracle's AdamW."""
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    theta = params.astype(np.float64)
    mm = np.zeros_like(theta)
    vv = np.zeros_like(theta)
    m.set_params(params)
    hg = _hgnn()
    db = hg.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    for t in range(1, 4):
        m.forward(db, pred)
        m.backward()
        g = m.grads().cpu().numpy().astype(np.float64)
        p0 = m.params().cpu().numpy().astype(np.float64)
        m.adam_step(lr=1e-3, weight_decay=0.01)
        p1 = m.params().cpu().numpy().astype(np.float64)
        ref, mm, vv = oracle.adamw(p0, g, mm, vv, t, lr=1e-3, weight_decay=0.01)
        r = rel(p1 - p0, ref - p0)
        say(f"  adam step {t}: update rel {r:.2e}")
        assert r <= 1e-5
        assert rel(p1, ref) <= 1e-6
    m.close()


def test_adam_steps_without_a_forward_between_them():
    """The weight copies and AdamW's step counter are refreshed by the next
    forward after a step; two steps in a row (no forward between them) must
    still count t = 1, 2, and a checkpoint taken before the refresh must hold
    the advanced count."""
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    m.set_params(params)
    hg = _hgnn()
    db = hg.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    m.forward(db, pred)
    m.backward()
    g = m.grads().cpu().numpy().astype(np.float64)
    theta = m.params().cpu().numpy().astype(np.float64)
    mm, vv = np.zeros_like(theta), np.zeros_like(theta)
    for t in (1, 2):
        m.adam_step(lr=1e-3, weight_decay=0.01)
        theta, mm, vv = oracle.adamw(theta, g, mm, vv, t, lr=1e-3, weight_decay=0.01)
        r = rel(m.params().cpu().numpy().astype(np.float64), theta)
        say(f"  step {t} without a forward: rel {r:.2e}")
        assert r <= 1e-6
    state = m.get_state()
    # the header ends with the step count (int64), then params, m, v follow
    hdr = state[:len(state) - 12 * m.num_params]
    assert int.from_bytes(hdr[-8:], "little", signed=True) == 2
    # a forward (which runs the refresh) leaves the count where it was
    m.forward(db, pred)
    assert m.get_state() == state
    m.close()


def test_checkpoint_resume_bitwise():
    hg = _hgnn()
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    db = hg.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")

    def steps(model, k):
        for _ in range(k):
            model.forward(db, pred)
            model.backward()
            model.adam_step()

    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    m.set_params(params)
    steps(m, 2)
    state = m.get_state()
    steps(m, 2)
    ref = m.params().clone()
    m2 = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    m2.set_state(state)
    steps(m2, 2)
    assert torch.equal(m2.params(), ref)
    m.close()
    m2.close()


# ---------------------------------------------------------------------------
# BF16 path
# ---------------------------------------------------------------------------

def test_bf16_outputs_within_2e2():
    w = synth.WORKLOADS["c2_train_bf16"]
    b, params = w.batch(), w.params()
    L, H = w.num_layers, w.hidden
    m = make_model(L, H, w.edge_feat, 1, 0, w.delta)
    out = run_train_step(m, b, params)
    rec = oracle.forward(params, b, L, H, w.delta)
    r_pred = rel(out["pred"].cpu().numpy(), rec.y)
    r_loss = rel([out["loss"].item()], [rec.loss])
    g_ref, _, stats = oracle.backward(rec, hint=gpu_decisions(m, L, H, b.num_nodes,
                                                              b.num_graphs), tau=TAU_BF16)
    rep = grad_report(m, out["grads"].cpu().numpy(), g_ref, w.shape)
    erep = grad_report(m, out["grads"].cpu().numpy(), g_ref, w.shape, elementwise=True)
    worst = max(rep, key=rep.get)
    e_pred = maxrel(out["pred"].cpu().numpy(), rec.y)
    say(f"bf16 c2: pred rel {r_pred:.2e} (element-wise {e_pred:.2e}) loss rel {r_loss:.2e}; "
        f"grad worst {worst} {rep[worst]:.2e} median {np.median(list(rep.values())):.2e}; "
        f"element-wise worst {max(erep.values()):.2e}; adopted {stats}")
    assert r_pred <= 2e-2 and r_loss <= 2e-2
    m.close()


C3_SAMPLE = list(range(0, 1024, 16))   # 64 graphs spread over the batch


def test_large_config_sampled_graphs():
    """8 layers, H=256, 1024 graphs, BF16 + recompute, the whole batch on the
    GPU: graphs are independent, so the oracle checks 64 of them; the
    per-operation path gives bitwise the same predictions."""
    w = synth.WORKLOADS["c3_large_bf16"]
    b, params = w.batch(), w.params()
    L, H = w.num_layers, w.hidden
    say(f"c3 full batch: N={b.num_nodes} E={b.num_edges}")
    m = make_model(L, H, w.edge_feat, 1, 1, w.delta)
    out = run_train_step(m, b, params)
    assert torch.isfinite(out["grads"]).all()
    # At this size the training path runs the message and update linears of
    # layers 1.. on BF16 copies of their inputs (the LDS-DMA kernel); the
    # per-operation path runs the register-staged kernel on the FP32 inputs.
    # Same roundings, same products in the same order: bitwise equal.
    net = _hgnn().PNANet(m, params)
    with torch.no_grad():
        p_ops = net(_hgnn().DeviceBatch.from_host(b))
    torch.cuda.synchronize()
    assert torch.equal(p_ops, out["pred"])
    say("  per-operation path (register-staged linears): predictions bitwise equal")
    pred = out["pred"].cpu().numpy()
    sub = synth.select_graphs(b, C3_SAMPLE)
    rec = oracle.forward(params, sub, L, H, w.delta)
    r = rel(pred[C3_SAMPLE], rec.y)
    say(f"  64 sampled graphs: pred rel {r:.2e} (element-wise "
        f"{maxrel(pred[C3_SAMPLE], rec.y):.2e})")
    assert r <= 2e-2
    m.close()


@pytest.mark.parametrize("H,recompute", [(64, 0), (192, 1)])
def test_bf16_copies_at_other_widths(H, recompute):
    """Batches of at least 16k nodes run the BF16 linears of layers 1.. on BF16
    copies of their inputs (LDS-DMA kernel, 128 x 128 tiles).  At H = 64 and
    192 the column tiles are partial (Ncols 64, 192, 384): the predictions
    equal the per-operation path's (register-staged kernel) bitwise, and
    sampled graphs match the FP64 oracle within the BF16 bound."""
    L = 3
    b = synth.make_batch(1009, 520, 10, 60, 1)
    assert b.num_nodes >= 16384
    params = synth.init_params(synth.ModelShape(L, H, 9, 1), 2009)
    say(f"H={H} recompute={recompute}: N={b.num_nodes} E={b.num_edges}")
    m = make_model(L, H, 1, 1, recompute, synth.DELTA_C1)
    out = run_train_step(m, b, params)
    assert torch.isfinite(out["grads"]).all()
    net = _hgnn().PNANet(m, params)
    with torch.no_grad():
        p_ops = net(_hgnn().DeviceBatch.from_host(b))
    torch.cuda.synchronize()
    assert torch.equal(p_ops, out["pred"])
    sample = [0, 1, 137, 260, 399, 519]
    rec = oracle.forward(params, synth.select_graphs(b, sample), L, H, synth.DELTA_C1)
    r = rel(out["pred"].cpu().numpy()[sample], rec.y)
    say(f"  bitwise equal to the per-operation path; sampled pred rel {r:.2e}")
    assert r <= 2e-2
    m.close()


def test_large_config_subbatch_loss_and_gradients():
    """The C3 model (8 layers, H=256, BF16 linears, recompute) on a 64-graph
    sub-batch of the C3 batch: predictions and loss within 2e-2 of the FP64
    oracle; the error of every gradient tensor reported, with the GPU's
    decisions replayed at tau = 3e-2 (the decisions are read from a model
    that stores every layer: its activations are bitwise those recomputed)."""
    w = synth.WORKLOADS["c3_large_bf16"]
    b, params = w.batch(), w.params()
    L, H = w.num_layers, w.hidden
    sub = synth.select_graphs(b, C3_SAMPLE)
    say(f"c3 sub-batch: B={sub.num_graphs} N={sub.num_nodes} E={sub.num_edges}")
    m = make_model(L, H, w.edge_feat, 1, 1, w.delta)
    out = run_train_step(m, sub, params)
    m2 = make_model(L, H, w.edge_feat, 1, 0, w.delta)
    o2 = run_train_step(m2, sub, params)
    assert torch.equal(o2["pred"], out["pred"])
    dec = gpu_decisions(m2, L, H, sub.num_nodes, sub.num_graphs)
    m2.close()
    rec = oracle.forward(params, sub, L, H, w.delta)
    pred = out["pred"].cpu().numpy()
    r_pred, r_loss = rel(pred, rec.y), rel([out["loss"].item()], [rec.loss])
    g_ref, _, stats = oracle.backward(rec, hint=dec, tau=TAU_BF16)
    g = out["grads"].cpu().numpy()
    rep = grad_report(m, g, g_ref, w.shape)
    erep = grad_report(m, g, g_ref, w.shape, elementwise=True)
    worst = max(rep, key=rep.get)
    say(f"  pred rel {r_pred:.2e} (element-wise {maxrel(pred, rec.y):.2e}) loss rel "
        f"{r_loss:.2e}; adopted {stats}")
    say(f"  gradient rel: worst {worst} {rep[worst]:.2e}, median "
        f"{np.median(list(rep.values())):.2e}; element-wise worst {max(erep.values()):.2e}")
    for l in range(L):
        say(f"    layer {l}: Wm {rep[f'l{l}.Wm']:.2e} bm {rep[f'l{l}.bm']:.2e} "
            f"Wp {rep[f'l{l}.Wp']:.2e} bp {rep[f'l{l}.bp']:.2e}")
    say(f"    head: W1 {rep['W1']:.2e} b1 {rep['b1']:.2e} w2 {rep['w2']:.2e} "
        f"b2 {rep['b2']:.2e}")
    assert r_pred <= 2e-2 and r_loss <= 2e-2
    assert np.all(np.isfinite(g))
    m.close()


# ---------------------------------------------------------------------------
# edge cases and malformed input
# ---------------------------------------------------------------------------

def test_edge_cases_empty_and_ragged():
    hg = _hgnn()
    shape = synth.ModelShape(2, 32, 9, 1)
    params = synth.init_params(shape, 9)
    rng = np.random.default_rng(0)
    # no edges at all: every node isolated (d = 0)
    b0 = synth.Batch(np.array([0, 1, 4], np.int32), rng.standard_normal((4, 9)).astype(np.float32),
                     np.zeros((2, 0), np.int32), np.zeros((0, 1), np.float32),
                     np.array([1.0, 2.0], np.float32))
    # single-node graphs mixed with ragged ones
    parts = [synth.make_batch(s, 1, n, n, 1) for s, n in [(1, 1), (2, 7), (3, 1), (4, 33)]]
    b1 = synth.concat_batches(parts)
    for b in (b0, b1):
        m = hg.Model(2, 32, 9, 1, 4, 0, 0, 1.0)
        out = run_train_step(m, b, params)
        rec = oracle.forward(params, b, 2, 32, 1.0)
        assert rel(out["pred"].cpu().numpy(), rec.y) <= 1e-5
        g_ref, _, _ = oracle.backward(rec, hint=gpu_decisions(m, 2, 32, b.num_nodes,
                                                              b.num_graphs), tau=TAU_FP32)
        assert rel(out["grads"].cpu().numpy(), g_ref) <= 1e-5
        m.close()


@pytest.mark.parametrize("kind", ["range", "cross", "degree", "empty"])
def test_malformed_batches_are_rejected(kind):
    hg = _hgnn()
    b = synth.make_batch(3, 3, 5, 8, 1)
    gp, ei = b.graph_ptr.copy(), b.edge_index.copy()
    if kind == "range":
        ei[0, 0] = b.num_nodes + 5
    elif kind == "cross":
        ei[0, 0] = b.num_nodes - 1
        ei[1, 0] = 0
    elif kind == "degree":
        pass
    elif kind == "empty":
        gp[1] = gp[0]
    bad = synth.Batch(gp, b.x, ei, b.edge_attr, b.y)
    m = hg.Model(1, 16, 9, 1, 1 if kind == "degree" else 4, 0, 0, 1.0)
    with pytest.raises(hg.HgnnError) as ei_:
        m.prepare(hg.DeviceBatch.from_host(bad), validate=True)
    assert ei_.value.code == hg.EINVAL
    # the context stays usable
    m.prepare(hg.DeviceBatch.from_host(b if kind != "degree" else
                                       synth.make_batch(3, 1, 2, 2, 1)), validate=True)
    m.close()


def test_deferred_validation_reports_through_check():
    """Without the validate flag a malformed batch runs to completion (the
    CSR builder skips bad edges, nothing reads out of bounds) and the error
    surfaces at the next check."""
    hg = _hgnn()
    b = synth.make_batch(4, 3, 5, 8, 1)
    ei = b.edge_index.copy()
    ei[0, 1] = b.num_nodes + 100
    bad = synth.Batch(b.graph_ptr, b.x, ei, b.edge_attr, b.y)
    m = hg.Model(2, 16, 9, 1, 4, 0, 0, 1.0)
    m.set_params(synth.init_params(synth.ModelShape(2, 16, 9, 1), 5))
    db = hg.DeviceBatch.from_host(bad)
    pred = torch.empty(bad.num_graphs, device="cuda")
    m.forward(db, pred)                     # no synchronisation, no error yet
    m.backward()
    with pytest.raises(hg.HgnnError) as e:
        m.check()
    assert e.value.code == hg.EINVAL and "out of range" in str(e.value)
    good = hg.DeviceBatch.from_host(b)
    m.forward(good, pred)
    m.check()                               # cleared by the next batch
    m.close()


# ---------------------------------------------------------------------------
# configuration sweep: hidden widths off the tile sizes, 0-4 edge features,
# degrees above the four in-edges a thread keeps in registers, recompute
# ---------------------------------------------------------------------------

def _dense_batch(seed, B, n_lo, n_hi, Fe, p_edge):
    """Random undirected graphs with edge probability p_edge (degrees well
    above a molecule's), both directions stored, bond-length-like features."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(n_lo, n_hi + 1, size=B)
    gp = np.concatenate([[0], np.cumsum(sizes)]).astype(np.int32)
    src, dst, attr = [], [], []
    for b in range(B):
        n, o = int(sizes[b]), int(gp[b])
        for i in range(n):
            for j in range(i + 1, n):
                if rng.random() < p_edge:
                    a = rng.uniform(0.9, 1.6, size=Fe)
                    src += [o + i, o + j]
                    dst += [o + j, o + i]
                    attr += [a, a]
    N = int(gp[-1])
    x = rng.standard_normal((N, 9)).astype(np.float32)
    ei = np.array([src, dst], np.int32).reshape(2, -1)
    ea = np.array(attr, np.float32).reshape(-1, Fe) if Fe else None
    y = rng.normal(5.0, 1.5, size=B).astype(np.float32)
    return synth.Batch(gp, x, ei, ea, y)


@pytest.mark.parametrize("L,H,Fe,maxd,recompute,p_edge", [
    (2, 16, 0, 16, 0, 0.8),     # complete-ish graphs: degrees up to 11
    (2, 48, 2, 16, 1, 0.5),     # H off the 64/128 tiles, two edge features, recompute
    (3, 32, 3, 8, 0, 0.4),
    (2, 80, 4, 12, 1, 0.6),     # four edge features
    (1, 512, 1, 16, 0, 0.5),    # the widest hidden size the header allows
])
def test_config_sweep_fp32_parity(L, H, Fe, maxd, recompute, p_edge):
    b = _dense_batch(1000 + H + Fe, 12, 3, 12, Fe, p_edge)
    deg = np.bincount(b.edge_index[1], minlength=b.num_nodes)
    assert deg.max() <= maxd
    shape = synth.ModelShape(L, H, 9, Fe)
    params = synth.init_params(shape, 77 + H)
    delta = 1.3
    say(f"sweep L={L} H={H} Fe={Fe} maxd={maxd} recompute={recompute}: N={b.num_nodes} "
        f"E={b.num_edges} max in-degree {deg.max()}")
    m = make_model(L, H, Fe, 0, recompute, delta, maxd=maxd)
    out = run_train_step(m, b, params)
    rec = oracle.forward(params, b, L, H, delta)
    r_pred = rel(out["pred"].cpu().numpy(), rec.y)
    r_loss = rel([out["loss"].item()], [rec.loss])
    if recompute:
        # decisions from the same forward with every layer stored (bitwise the
        # same activations; a separate test checks that)
        m2 = make_model(L, H, Fe, 0, 0, delta, maxd=maxd)
        run_train_step(m2, b, params, backward=False)
        dec = gpu_decisions(m2, L, H, b.num_nodes, b.num_graphs)
        m2.close()
    else:
        dec = gpu_decisions(m, L, H, b.num_nodes, b.num_graphs)
    g_ref, _, stats = oracle.backward(rec, hint=dec, tau=TAU_FP32)
    rep = grad_report(m, out["grads"].cpu().numpy(), g_ref, shape)
    worst = max(rep, key=rep.get)
    say(f"  pred rel {r_pred:.2e} loss rel {r_loss:.2e}; worst grad {worst} {rep[worst]:.2e}; "
        f"adopted {stats}")
    assert r_pred <= 1e-5 and r_loss <= 1e-5
    for k, v in rep.items():
        assert v <= 1e-5, (k, v)
    m.close()


def test_param_views_alias_the_context_vectors():
    """hgnn_param_views: the gradient view holds what hgnn_get_grads copies;
    a write through the parameter view reaches the layers after
    set_params(view), which then copies nothing."""
    from paper_2207_11333_amd import hgnn
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    out = run_train_step(m, b, params)
    pv, gv = m.param_views()
    p_t, g_t = pv.tensor(), gv.tensor()
    assert torch.equal(g_t, out["grads"]) and torch.equal(p_t, m.params())
    p_t.mul_(0.5)                                   # in place, through the view
    m.set_params(pv)
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    m.forward(db, pred)
    m2 = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    m2.set_params(params * 0.5)
    pred2 = torch.empty(b.num_graphs, device="cuda")
    m2.forward(db, pred2)
    torch.cuda.synchronize()
    assert torch.equal(pred, pred2)
    m.close()
    m2.close()


def test_same_step_on_another_stream_is_bitwise_equal():
    """The library runs on whatever stream the caller passes: the same
    training step on a side stream gives bitwise the same outputs."""
    hg = _hgnn()
    w = synth.WORKLOADS["c0_small_fp32"]
    b, params = w.batch(), w.params()
    db = hg.DeviceBatch.from_host(b)
    outs = []
    for use_side in (False, True):
        m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
        m.set_params(params)
        pred = torch.empty(b.num_graphs, device="cuda")
        loss = torch.empty(1, device="cuda")
        side = torch.cuda.Stream()
        side.wait_stream(torch.cuda.current_stream())
        with torch.cuda.stream(side if use_side else torch.cuda.current_stream()):
            m.forward(db, pred, loss)
            m.backward()
            m.adam_step()
            p = m.params()
        torch.cuda.synchronize()
        outs.append((pred, loss, p))
        m.close()
    for a, c in zip(outs[0], outs[1]):
        assert torch.equal(a, c)


# ---------------------------------------------------------------------------
# boundary: seeded initialisation, stale backward refused
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("kind", ["pna", "sage", "cgcnn"])
def test_seeded_init_matches_its_definition(kind):
    """hgnn_create with no init_params (PNA) and hgnn_init_params (any kind)
    give bit for bit the host-side SplitMix64 + Xavier definition."""
    hg = _hgnn()
    L, H, Fe = 2, 32, 1
    if kind == "pna":
        shapes = synth.ModelShape(L, H, 9, Fe).tensor_shapes()
        m = hg.Model(L, H, 9, Fe, 4, 0, 0, 1.0, seed=1234)
        got = m.params().cpu().numpy()
        ref = synth.counter_init_params(shapes, 1234)
        assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
        # explicit initial parameters are copied as given
        p = synth.init_params(synth.ModelShape(L, H, 9, Fe), 5)
        m2 = hg.Model(L, H, 9, Fe, 4, 0, 0, 1.0, init_params=p)
        assert np.array_equal(m2.params().cpu().numpy(), p)
        m2.close()
    else:
        shapes = synth.gc_tensor_shapes(kind, L, H, 9, Fe)
        m = hg.Model(L, H, 9, Fe, 4, 0, 0, 1.0, kind=kind)
    m.init_params(99)
    got = m.params().cpu().numpy()
    ref = synth.counter_init_params(shapes, 99)
    assert np.array_equal(got.view(np.uint32), ref.view(np.uint32))
    m.close()


def test_backward_of_a_superseded_forward_is_refused():
    """Two forwards before one backward: the first one's stored state is gone,
    so its backward must fail loudly instead of using the second batch."""
    hg = _hgnn()
    w = synth.WORKLOADS["c0_small_fp32"]
    b1, params = w.batch(), w.params()
    b2 = synth.make_batch(555, 80, 5, 30, w.edge_feat)   # more nodes than b1
    m = make_model(w.num_layers, w.hidden, w.edge_feat, 0, 0, w.delta)
    net = hg.PNANet(m, params)
    d1, d2 = hg.DeviceBatch.from_host(b1), hg.DeviceBatch.from_host(b2)
    p1 = net(d1)
    p2 = net(d2)
    with pytest.raises(hg.HgnnError) as e:
        ((p1 - d1.y) ** 2).mean().backward()
    assert e.value.code == hg.EINVAL and "generation" in str(e.value)
    ((p2 - d2.y) ** 2).mean().backward()            # the live one still works
    torch.cuda.synchronize()
    assert torch.isfinite(net.packed_grad()).all()
    # the fused entry points through ModelFunction
    gnet = hg.GCNet(m, params)
    q1 = gnet(d1)
    q2 = gnet(d2)
    with pytest.raises(hg.HgnnError):
        q1.sum().backward()
    q2.sum().backward()
    m.close()
