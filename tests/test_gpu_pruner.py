"""GPU pruner kernels (bf16 MFMA, fp32 accumulate) against the FP64 CPU twin."""
import numpy as np
import pytest
import torch

import mlp
from paper_2405_13409_amd import scenes

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def sp():
    from paper_2405_13409_amd import spoly

    spoly.load_library()
    return spoly


@pytest.fixture(scope="module")
def ctx(sp):
    c = sp.Context(0)
    yield c
    c.close()


def _batch(n, seed):
    mesh = scenes.caustic_sphere()
    R = scenes.caustic_receivers()
    x3 = scenes.CAUSTIC_LIGHT_OUTSIDE
    rng = np.random.default_rng(seed)
    q0 = rng.integers(0, len(R), n).astype(np.int32)
    q3 = np.zeros(n, dtype=np.int32)
    qt = rng.integers(0, mesh.nt, (n, 2)).astype(np.int32)
    y = (rng.random(n) < 0.1).astype(np.float32)
    return mesh, R, x3, q0, q3, qt, y


def _dev(sp, mesh, R, x3, q0, q3, qt):
    t = lambda a: torch.from_numpy(np.ascontiguousarray(a)).cuda()  # noqa: E731
    return sp.DeviceMesh(mesh.P, mesh.N, mesh.tri), sp.DevicePoints(R), sp.DevicePoints(x3), t(q0), t(q3), t(qt)


def test_features_match_twin(sp, ctx):
    print("[gpu-case] pruner features", flush=True)
    mesh, R, x3, q0, q3, qt, y = _batch(1000, 1)
    dm, dR, d3, t0, t3, tt = _dev(sp, mesh, R, x3, q0, q3, qt)
    f = ctx.pruner_features(dm, dR, d3, t0, t3, tt).cpu().numpy()
    ref = mlp.features(mesh.P, mesh.N, mesh.tri, R, x3, q0, q3, qt)
    assert np.allclose(f[:, :42], ref.astype(np.float32), rtol=0, atol=1e-7)
    assert np.all(f[:, 42:] == 0)


@pytest.mark.parametrize("n,tol", [(4096, 2e-2), (16384, 2e-2), (100, 6e-2)])
def test_forward_backward_vs_fp64_twin(sp, ctx, n, tol):
    """bf16 operands carry 8 mantissa bits; at the training batch sizes the
    per-tensor relative gradient error stays below 2e-2, at a tiny batch the
    cancellation in the sums allows a few per cent."""
    print(f"[gpu-case] pruner fwd/bwd n={n}", flush=True)
    mesh, R, x3, q0, q3, qt, y = _batch(n, 2)
    dm, dR, d3, t0, t3, tt = _dev(sp, mesh, R, x3, q0, q3, qt)
    p = mlp.init_params(3)
    X = mlp.features(mesh.P, mesh.N, mesh.tri, R, x3, q0, q3, qt)
    # the GPU sees bf16 inputs and weights: compare against the twin on the same rounded values
    bf = lambda a: torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()  # noqa: E731
    loss_ref, g_ref = mlp.loss_and_grad(p, bf(X), y.astype(np.float64), 5.0)
    params = torch.from_numpy(p.astype(np.float32)).cuda()
    grads = torch.zeros_like(params)
    loss = torch.zeros(1, dtype=torch.float32, device="cuda")
    ctx.pruner_fwd_bwd(dm, dR, d3, t0, t3, tt, torch.from_numpy(y).cuda(), 5.0, params, grads, loss)
    torch.cuda.synchronize()
    g = grads.cpu().numpy().astype(np.float64)
    assert abs(loss.item() - loss_ref) <= 2e-2 * abs(loss_ref)
    G, Gr = mlp.unpack(g), mlp.unpack(g_ref)
    for name, _ in mlp.SIZES:
        a, b = G[name].ravel(), Gr[name].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        print(name, rel)
        assert rel <= tol, (name, rel)


def test_score_kernel_vs_twin(sp, ctx):
    print("[gpu-case] pruner score", flush=True)
    mesh, R, x3, q0, q3, qt, y = _batch(5000, 4)
    dm, dR, d3, t0, t3, tt = _dev(sp, mesh, R, x3, q0, q3, qt)
    p = mlp.init_params(5)
    X = mlp.features(mesh.P, mesh.N, mesh.tri, R, x3, q0, q3, qt)
    z, _ = mlp.forward(p, X)
    pref = 1 / (1 + np.exp(-z))
    params = torch.from_numpy(p.astype(np.float32)).cuda()
    scores = torch.zeros(len(q0), dtype=torch.float32, device="cuda")
    thr = float(np.median(pref))
    keep, kc = ctx.prune_score(dm, dR, d3, t0, t3, tt, params, thr, scores=scores)
    torch.cuda.synchronize()
    s = scores.cpu().numpy()
    assert np.max(np.abs(s - pref)) < 3e-2
    kept = np.sort(keep[: int(kc.item())].cpu().numpy())
    assert np.array_equal(kept, np.nonzero(s >= thr)[0])


def test_adam_step_matches_reference(sp, ctx):
    print("[gpu-case] adam", flush=True)
    rng = np.random.default_rng(6)
    p = rng.normal(size=mlp.NPARAMS).astype(np.float32)
    g = rng.normal(size=mlp.NPARAMS).astype(np.float32)
    P, G = torch.from_numpy(p.copy()).cuda(), torch.from_numpy(g).cuda()
    m, v = torch.zeros_like(P), torch.zeros_like(P)
    for step in (1, 2):
        ctx.pruner_step(P, G, m, v, step, 1e-3, 0.9, 0.999, 1e-8)
    torch.cuda.synchronize()
    mm, vv, pp = np.zeros_like(p, dtype=np.float64), np.zeros_like(p, dtype=np.float64), p.astype(np.float64)
    for step in (1, 2):
        mm = 0.9 * mm + 0.1 * g
        vv = 0.999 * vv + 0.001 * g.astype(np.float64) ** 2
        pp = pp - 1e-3 * (mm / (1 - 0.9 ** step)) / (np.sqrt(vv / (1 - 0.999 ** step)) + 1e-8)
    assert np.max(np.abs(P.cpu().numpy() - pp)) < 1e-5


def _bf16(a):
    """Round to bfloat16 (nearest even) through float32, as the kernel does."""
    return torch.from_numpy(np.asarray(a, dtype=np.float32)).to(torch.bfloat16).to(torch.float64).numpy()


def _forward_bf16(p, X):
    """FP64 twin forward with the kernel's roundings: inputs, weights and each
    hidden layer's activations rounded to bf16; biases in float32."""
    W = mlp.unpack(p)
    b = {k: np.asarray(W[k], dtype=np.float32).astype(np.float64) for k in ("b1", "b2", "b3", "b4")}
    h = _bf16(X)
    for i in (1, 2, 3):
        h = _bf16(np.maximum(h @ _bf16(W[f"W{i}"]) + b[f"b{i}"], 0.0))
    return h @ _bf16(W["W4"]) + b["b4"][0]


@pytest.mark.parametrize("weights,n", [("init", 20007), ("trained", 20007), ("init", 5)])
def test_score_kernel_vs_bf16_twin(sp, ctx, weights, n):
    """Against a twin that rounds where the kernel rounds, only the order of
    the fp32 sums differs (and with it, rarely, one activation's bf16
    rounding), so the scores agree far inside the plain twin's bound; the
    batch spans many 16-tuple tiles and a ragged last one."""
    print(f"[gpu-case] pruner score bf16 twin {weights} n={n}", flush=True)
    mesh, R, x3, q0, q3, qt, y = _batch(n, 6)
    dm, dR, d3, t0, t3, tt = _dev(sp, mesh, R, x3, q0, q3, qt)
    if weights == "init":
        p = mlp.init_params(7)
    else:
        from paper_2405_13409_amd import train_pruner

        p = train_pruner.load().params.cpu().numpy().astype(np.float64)
    X = mlp.features(mesh.P, mesh.N, mesh.tri, R, x3, q0, q3, qt)
    z = _forward_bf16(p, X)
    pref = 1 / (1 + np.exp(-z))
    params = torch.from_numpy(p.astype(np.float32)).cuda()
    scores = torch.zeros(len(q0), dtype=torch.float32, device="cuda")
    ctx.prune_score(dm, dR, d3, t0, t3, tt, params, 0.5, scores=scores)
    torch.cuda.synchronize()
    d = np.abs(scores.cpu().numpy() - pref)
    print("max", d.max(), "median", np.median(d))
    assert d.max() < 2e-3 and np.median(d) < 1e-5


def test_weight_gradients_repeat_bitwise(sp, ctx):
    """The weight gradients of a large batch are summed over up to 128 split-K
    partial tiles in a fixed order, without atomics: two passes give the same
    bits, and the result still agrees with the FP64 twin.  The reported loss
    is summed with atomics, so it agrees only to rounding."""
    n = 65536
    print(f"[gpu-case] pruner split-K repeat n={n}", flush=True)
    mesh, R, x3, q0, q3, qt, y = _batch(n, 8)
    dm, dR, d3, t0, t3, tt = _dev(sp, mesh, R, x3, q0, q3, qt)
    p = mlp.init_params(9)
    params = torch.from_numpy(p.astype(np.float32)).cuda()
    yt = torch.from_numpy(y).cuda()
    out = []
    for _ in range(2):
        grads = torch.zeros_like(params)
        loss = torch.zeros(1, dtype=torch.float32, device="cuda")
        ctx.pruner_fwd_bwd(dm, dR, d3, t0, t3, tt, yt, 5.0, params, grads, loss)
        torch.cuda.synchronize()
        out.append((grads.cpu().numpy(), float(loss.item())))
    assert out[0][0].tobytes() == out[1][0].tobytes()
    assert abs(out[0][1] - out[1][1]) <= 1e-5 * abs(out[0][1])
    X = mlp.features(mesh.P, mesh.N, mesh.tri, R, x3, q0, q3, qt)
    bf = lambda a: torch.from_numpy(a.astype(np.float32)).to(torch.bfloat16).to(torch.float64).numpy()  # noqa: E731
    _, g_ref = mlp.loss_and_grad(p, bf(X), y.astype(np.float64), 5.0)
    G, Gr = mlp.unpack(out[0][0].astype(np.float64)), mlp.unpack(g_ref)
    for name in ("W1", "W2", "W3", "W4"):
        a, b = G[name].ravel(), Gr[name].ravel()
        rel = np.linalg.norm(a - b) / max(np.linalg.norm(b), 1e-30)
        assert rel <= 2e-2, (name, rel)
