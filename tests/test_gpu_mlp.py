"""GPU parity of the cost model's network kernels against the FP64 oracle:
logits, loss and every gradient tensor within 1e-5 relative (norm), and one
Adam step within 1e-5 relative.
"""
import numpy as np
import pytest
import torch

import oracle

pytestmark = pytest.mark.gpu

DIMS = (16, 64, 64, 48)


def _params(g, F, H1, H2, K):
    return {"W1": g.standard_normal((H1, F)) * 0.4, "b1": g.standard_normal(H1) * 0.1,
            "W2": g.standard_normal((H2, H1)) * 0.2, "b2": g.standard_normal(H2) * 0.1,
            "W3": g.standard_normal((K, H2)) * 0.2, "b3": g.standard_normal(K) * 0.1}


def _flat(P):
    return np.concatenate([P[k].ravel() for k in ("W1", "b1", "W2", "b2", "W3", "b3")])


def _rel(a, b):
    return np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)


@pytest.mark.parametrize("B", [1, 7, 256, 4096])
def test_loss_grad_vs_oracle(gpu_lib, B):
    om = gpu_lib
    F, H1, H2, K = DIMS
    g = np.random.Generator(np.random.PCG64(B))
    P = _params(g, F, H1, H2, K)
    P32 = {k: v.astype(np.float32) for k, v in P.items()}
    X = g.standard_normal((B, F)).astype(np.float32)
    y = g.integers(0, K, B).astype(np.int32)
    loss_ref, Z_ref, g_ref = oracle.mlp_loss_grad(X.astype(np.float64), y,
                                                  {k: v.astype(np.float64) for k, v in P32.items()})
    params = torch.from_numpy(_flat(P32)).cuda()
    assert params.numel() == om.mlp_param_count(*DIMS)
    Xd = torch.from_numpy(X).cuda()
    yd = torch.from_numpy(y).cuda()
    Z = torch.zeros((B, K), dtype=torch.float32, device="cuda")
    om.mlp_forward(DIMS, params, Xd, Z)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    grads = torch.zeros_like(params)
    om.mlp_loss_grad(DIMS, params, Xd, yd, loss, grads)
    torch.cuda.synchronize()
    assert _rel(Z.cpu().numpy().astype(np.float64), Z_ref) < 1e-5
    assert abs(loss.item() - loss_ref) <= 1e-5 * abs(loss_ref)
    gh = grads.cpu().numpy().astype(np.float64)
    off = 0
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        sz = g_ref[k].size
        assert _rel(gh[off:off + sz], g_ref[k].ravel()) < 1e-5, k
        off += sz


def test_adam_vs_oracle(gpu_lib):
    om = gpu_lib
    g = np.random.Generator(np.random.PCG64(3))
    n = 10_000
    w = g.standard_normal(n).astype(np.float32)
    m = (g.standard_normal(n) * 0.01).astype(np.float32)
    v = np.abs(g.standard_normal(n) * 0.001).astype(np.float32)
    gr = g.standard_normal(n).astype(np.float32)
    wd, md, vd, gd = (torch.from_numpy(a.copy()).cuda() for a in (w, m, v, gr))
    om.mlp_adam(wd, md, vd, gd, 7, lr=1e-2)
    torch.cuda.synchronize()
    # the kernel receives fp32 hyperparameters: give the oracle the same values
    f32 = lambda v: float(np.float32(v))
    w2, m2, v2 = oracle.adam(w, m, v, gr, 7, lr=f32(1e-2), beta1=f32(0.9), beta2=f32(0.999),
                             eps=f32(1e-8))
    assert _rel(wd.cpu().numpy(), w2) < 1e-6
    assert _rel(md.cpu().numpy(), m2) < 1e-6
    assert _rel(vd.cpu().numpy(), v2) < 1e-6


def test_adam_counted_equals_adam(gpu_lib):
    """The step number in device memory gives the update of omprt_mlp_adam at that step,
    bit for bit, and advances the counter by one per call."""
    om = gpu_lib
    g = np.random.Generator(np.random.PCG64(3))
    n = 9000
    p = torch.from_numpy(g.standard_normal(n).astype(np.float32)).cuda()
    a = [p.clone(), torch.zeros_like(p), torch.zeros_like(p)]
    b = [p.clone(), torch.zeros_like(p), torch.zeros_like(p)]
    step = torch.zeros(1, dtype=torch.int32, device="cuda")
    for t in range(1, 6):
        grads = torch.from_numpy(g.standard_normal(n).astype(np.float32)).cuda()
        om.mlp_adam(a[0], a[1], a[2], grads, t, lr=1e-2)
        om.mlp_adam_counted(b[0], b[1], b[2], grads, step, lr=1e-2)
        torch.cuda.synchronize()
        for u, w in zip(a, b):
            assert torch.equal(u.view(torch.int32), w.view(torch.int32)), t
        assert int(step.item()) == t


def test_training_graph_replays_match_eager(gpu_lib):
    """One epoch of training steps captured in a HIP graph and replayed every epoch
    (with the epoch's permutation done eagerly between replays) makes the same
    parameters, bit for bit, as the steps launched one by one and as the plain loop
    that copies every batch from the host and reads every loss back."""
    from paper_2106_03219_amd import train as tr
    om = gpu_lib
    g = np.random.Generator(np.random.PCG64(11))
    X = g.standard_normal((1000, 16)).astype(np.float32)
    y = g.integers(0, tr.DIMS[3], 1000).astype(np.int32)
    out = {}
    for mode in ("sync", "eager", "graph"):
        logs = []
        p = tr.train(om, torch, X, y, epochs=4, batch=96, lr=1e-3, seed=5, mode=mode,
                     log=logs.append)
        out[mode] = (p.cpu().numpy(), logs)
    for mode in ("eager", "graph"):
        assert np.array_equal(out[mode][0].view(np.uint32), out["sync"][0].view(np.uint32)), mode
    assert out["graph"][1][-1].split()[-1] == out["eager"][1][-1].split()[-1]
