"""The allocation-free inference forward (hgnn_forward_noalloc) against the
forward it is a variant of (hgnn_forward), through the C-ABI: two calls in a
row, the second on a smaller batch, in FP32 (1e-5 relative, the FP32 bar)
and BF16 (2e-2 relative on the outputs, the BF16 bar), plus the refusal of a
batch whose workspace exceeds the static array."""
import ctypes
import sys

import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2207_11333_amd import synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


def rel(a, r):
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.linalg.norm(a - r) / max(np.linalg.norm(r), 1e-30))


def maxrel(a, r):
    a = np.asarray(a, np.float64)
    r = np.asarray(r, np.float64)
    return float(np.abs(a - r).max() / max(np.abs(r).max(), 1e-30))


@pytest.mark.parametrize("prec,tol", [(0, 1e-5), (1, 2e-2)])
def test_noalloc_forward_matches_forward(prec, tol):
    from paper_2207_11333_amd import hgnn
    w = synth.WORKLOADS["c1_train_fp32"]
    m = hgnn.Model(w.num_layers, w.hidden, 9, w.edge_feat, 4, prec, 0, w.delta)
    m.set_params(w.params())
    # the first call on the full C1-shaped batch, the second on a smaller one
    big = synth.make_batch(w.data_seed, w.num_graphs, w.n_lo, w.n_hi, w.edge_feat)
    small = synth.make_batch(w.data_seed + 7, 24, w.n_lo, w.n_hi, w.edge_feat)
    for name, b in (("first", big), ("second, smaller", small)):
        say(f"noalloc prec={prec} {name}: B={b.num_graphs} N={b.num_nodes} E={b.num_edges}, "
            f"workspace {m.noalloc_bytes(b.num_graphs, b.num_nodes, b.num_edges)} bytes")
        db = hgnn.DeviceBatch.from_host(b)
        p_ref = torch.empty(b.num_graphs, device="cuda")
        l_ref = torch.empty(1, device="cuda")
        p_na = torch.full((b.num_graphs,), float("nan"), device="cuda")
        l_na = torch.full((1,), float("nan"), device="cuda")
        m.forward(db, p_ref, l_ref, validate=True)
        m.forward_noalloc(db, p_na, l_na, validate=True)
        torch.cuda.synchronize()
        a, r = p_na.cpu().numpy(), p_ref.cpu().numpy()
        e_pred, e_el = rel(a, r), maxrel(a, r)
        e_loss = abs(l_na.item() - l_ref.item()) / abs(l_ref.item())
        say(f"  pred rel {e_pred:.2e} (element-wise {e_el:.2e}), loss rel {e_loss:.2e}")
        assert np.all(np.isfinite(a))
        assert e_pred <= tol and e_el <= tol and e_loss <= tol
    # the training state was left alone: a backward of the last hgnn_forward
    # still runs
    m.backward()
    torch.cuda.synchronize()
    m.close()


def test_noalloc_refuses_oversized_batch():
    from paper_2207_11333_amd import hgnn
    w = synth.WORKLOADS["c1_train_fp32"]
    m = hgnn.Model(w.num_layers, w.hidden, 9, w.edge_feat, 4, 0, 0, w.delta)
    limit = int(hgnn.lib().hgnn_noalloc_max_bytes())
    b = synth.make_batch(w.data_seed, 512, 40, 60, w.edge_feat)
    need = m.noalloc_bytes(b.num_graphs, b.num_nodes, b.num_edges)
    say(f"oversized: N={b.num_nodes} needs {need} bytes of {limit}")
    assert need > limit
    db = hgnn.DeviceBatch.from_host(b)
    pred = torch.empty(b.num_graphs, device="cuda")
    with pytest.raises(hgnn.HgnnError) as ei:
        m.forward_noalloc(db, pred)
    assert ei.value.code == hgnn.EINVAL and "workspace" in str(ei.value)
    # the context is still usable
    small = synth.make_batch(w.data_seed, 8, w.n_lo, w.n_hi, w.edge_feat)
    ds = hgnn.DeviceBatch.from_host(small)
    p = torch.empty(8, device="cuda")
    m.forward_noalloc(ds, p)
    torch.cuda.synchronize()
    assert np.all(np.isfinite(p.cpu().numpy()))
    m.close()
