"""GPU parity of the learned proposal's network and features against the
numpy FP64 oracle (oracle/mdn.py) and the C oracle's feature builders.

Tolerances.  The GPU multiplies BF16 operands exactly into FP32
accumulators; the oracle rounds to BF16 at the same places and accumulates
in FP64.  What remains is FP32 accumulation order (relative 1e-6) and BF16
re-rounding of hidden activations and backpropagated gradients whose FP32
values land on the other side of a rounding boundary (one BF16 ulp, 2^-8
relative, for a small fraction of entries).  Over 256-long dot products
those flips average out to about 2^-8 / sqrt(256) of the output scale, so
head outputs agree to 1e-2 of their RMS; gradients are bounded element by
element by the BF16 flip bound taken from the oracle's absolute-value
products.
"""
import numpy as np
import pytest

import oracle as O
from oracle import mdn as D
from paper_1612_00595_amd import workloads as W

from gpu_cases import dynamic_small, instance, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def torch_dev():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_dev_bf16(torch, X):
    return torch.from_numpy(np.ascontiguousarray(X, dtype=np.float32)).to("cuda").to(torch.bfloat16)


def random_params(seed, scale=0.06):
    rng = np.random.default_rng(seed)
    lay, n = D.param_layout()
    flat = rng.normal(0, scale, n).astype(np.float32)
    P = D.unflatten(flat.astype(np.float64))
    P["W4"][56:] = 0.0
    P["b4"][56:] = 0.0
    P["b4"][4:56:7] -= 1.0          # log sds start inside their clamps
    flat = D.flatten(P).astype(np.float32)
    return flat, D.unflatten(flat.astype(np.float64))


def oracle_pairs(seed, first, count, spec=W.SMALL.model):
    m = O.make_model(**spec.asdict())
    F, T = D.pairs(m, seed, first, count)
    return D.to_bf16(F), D.to_f32(T)


def test_mdn_param_roundtrip_and_init(torch_dev):
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    say("[mdn] init / set / get")
    net = chromh.MDN(seed=7)
    P = D.unflatten(net.get_params().astype(np.float64))
    for l, (fi, fo) in enumerate(D.LAYERS):
        Wl = P[f"W{l + 1}"]
        live = 56 if l == 3 else fo
        a = np.sqrt(6.0 / (fi + live))
        assert np.all(np.abs(Wl[:live]) <= a) and np.all(Wl[live:] == 0)
        # U(-a, a): variance a^2 / 3
        assert np.var(Wl[:live]) == pytest.approx(a * a / 3, rel=0.05)
        assert np.all(P[f"b{l + 1}"] == 0)
    flat, _ = random_params(1)
    net.set_params(flat)
    assert np.array_equal(net.get_params(), flat)
    torch.cuda.synchronize()


# Element-wise bar for BF16 head outputs: each hidden activation the GPU
# rounds to BF16 can sit one rounding step (relative 2^-8) from the oracle's
# when the FP32 and FP64 pre-activations straddle a rounding boundary; such
# flips reach head output (m, i) through |a_mj| |W4_ij|, so the output moves
# by at most a few steps of (|A3| |W4|^T)_mi (flips in earlier layers reach
# it damped through the same product).
HEAD_ULPS = 4.0


def head_bound(As, Ws):
    return HEAD_ULPS * 2.0 ** -8 * (np.abs(As[3]) @ np.abs(Ws[3]).T) + 1e-9


@pytest.mark.parametrize("rows", [1, 300])
def test_mdn_forward_matches_oracle(torch_dev, rows):
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    say(f"[mdn] forward rows={rows}")
    flat, P = random_params(2)
    X, _ = oracle_pairs(11, 0, rows)
    net = chromh.MDN(seed=None)
    net.set_params(flat)
    out = net.forward(to_dev_bf16(torch, X)).cpu().numpy().astype(np.float64)
    ref, _, As, Ws = D.forward(P, X, bf16=True)
    assert np.all(out[:, 56:] == 0.0)
    ratio = np.abs(out - ref) / head_bound(As, Ws)
    say(f"[mdn] worst head element at {ratio.max():.3f} of its bound")
    assert np.all(ratio <= 1.0)


@pytest.mark.parametrize("rows", [1, 300, 1000])
def test_mdn_fused_inference_matches_oracle_and_forward(torch_dev, rows):
    """The fused inference kernel (tiles of 128 rows, ragged last tile) gives
    the oracle's head within the forward's tolerance and the layer-by-layer
    forward's values (the same BF16 activations and MFMA order)."""
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    say(f"[mdn] fused inference rows={rows}")
    flat, P = random_params(4)
    X, _ = oracle_pairs(13, 0, rows)
    net = chromh.MDN(seed=None)
    net.set_params(flat)
    Xd = to_dev_bf16(torch, X)
    got = net.infer(Xd).cpu().numpy().astype(np.float64)
    fwd = net.forward(Xd).cpu().numpy().astype(np.float64)
    ref, _, As, Ws = D.forward(P, X, bf16=True)
    scale = np.sqrt(np.mean(ref[:, :56] ** 2))
    ratio = np.abs(got - ref) / head_bound(As, Ws)
    say("[mdn] max abs error: fused", np.abs(got - ref).max(), "layer by layer",
        np.abs(fwd - ref).max(), "fused - layer by layer", np.abs(got - fwd).max(),
        "scale", scale, f"worst element at {ratio.max():.3f} of its bound")
    assert np.all(got[:, 56:] == 0.0)
    assert np.allclose(got, fwd, rtol=1e-5, atol=1e-5 * scale)
    assert np.all(ratio <= 1.0)


# Element-wise bar for BF16 gradients: the GPU rounds the output gradient,
# the hidden-layer gradients and the activations to BF16 (as the oracle does
# in its bf16 mode) but accumulates in FP32 where the oracle uses FP64, so an
# operand can sit one BF16 rounding step (relative 2^-8) away from the
# oracle's; through the product of two such operands, and the backward chain
# of layers above, a gradient element then moves by at most a few of those
# steps of its absolute-value product |dH|^T |A| (|dH| summed for a bias).
GRAD_ULPS = 4.0


@pytest.mark.parametrize("rows", [200, 2080])
def test_mdn_gradients_match_oracle(torch_dev, rows):
    """200 rows: one split of the batch reduction; 2 080 rows: five splits,
    their partial products and column sums summed by the job launch."""
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    say(f"[mdn] gradients rows={rows}")
    flat, P = random_params(3)
    X, Z = oracle_pairs(12, 500, rows)
    net = chromh.MDN(seed=None)
    net.set_params(flat)
    loss, grad = net.gradients(to_dev_bf16(torch, X),
                               torch.from_numpy(Z.astype(np.float32)).cuda())
    loss = loss.cpu().numpy().astype(np.float64)
    G = D.unflatten(grad.cpu().numpy().astype(np.float64))
    mean, per_row, Gref, ops = D.loss_and_grads(P, X, Z, bf16=True, parts=True)
    assert np.allclose(loss, per_row, rtol=1e-3, atol=1e-3 * np.abs(per_row).mean())
    for l in (4, 3, 2, 1):
        dH, A = ops[l]
        for name, bound in ((f"W{l}", np.abs(dH).T @ np.abs(A)), (f"b{l}", np.abs(dH).sum(0))):
            g, r = G[name], Gref[name]
            tol = GRAD_ULPS * 2.0 ** -8 * bound + 1e-12
            ratio = np.abs(g - r) / tol
            say(f"[mdn]   {name}: |g| {np.linalg.norm(r):.3e}, worst element at "
                f"{ratio.max():.3f} of its bound")
            assert np.all(ratio <= 1.0), name
    assert np.all(G["W4"][56:] == 0) and np.all(G["b4"][56:] == 0)


def test_mdn_clamped_log_sd_has_no_gradient(torch_dev):
    """Log sds beyond their clamp carry no gradient: with component 2's
    log-sd biases far above the upper clamp and component 5's far below the
    lower one for every row, those head outputs' weight and bias gradients
    are exactly zero on the GPU (and in the oracle), while the other
    outputs' are not."""
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    rows = 128
    flat, P = random_params(5)
    for d in range(3):
        P["b4"][7 * 2 + 4 + d] = 50.0
        P["b4"][7 * 5 + 4 + d] = -50.0
    flat = D.flatten(P)
    X, Z = oracle_pairs(14, 100, rows)
    net = chromh.MDN(seed=None)
    net.set_params(flat)
    _, grad = net.gradients(to_dev_bf16(torch, X), torch.from_numpy(Z.astype(np.float32)).cuda())
    G = D.unflatten(grad.cpu().numpy().astype(np.float64))
    _, _, Gref = D.loss_and_grads(P, X, Z, bf16=True)
    clamped = [7 * k + 4 + d for k in (2, 5) for d in range(3)]
    for o in clamped:
        assert np.all(G["W4"][o] == 0.0) and G["b4"][o] == 0.0, o
        assert np.all(Gref["W4"][o] == 0.0) and Gref["b4"][o] == 0.0, o
    free = [7 * k + 4 + d for k in (0, 1, 3) for d in range(3)]
    assert all(np.any(G["W4"][o] != 0.0) for o in free)


def test_mdn_adam_step_matches_oracle(torch_dev):
    """One Adam step (from zero moments: w - lr g / (|g| + eps)) on the
    oracle's gradients; entries whose oracle gradient is small against the
    GPU/oracle gradient disagreement may differ in sign and are skipped."""
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    rows, lr = 128, 1e-3
    say("[mdn] adam step")
    flat, P = random_params(4)
    X, Z = oracle_pairs(13, 900, rows)
    net = chromh.MDN(seed=None)
    net.set_params(flat)
    net.train_step(to_dev_bf16(torch, X), torch.from_numpy(Z.astype(np.float32)).cuda(), 1, lr)
    after = D.unflatten(net.get_params().astype(np.float64))
    _, _, Gref = D.loss_and_grads(P, X, Z, bf16=True)
    checked = 0
    for name, g in Gref.items():
        want = P[name] - lr * g / (np.abs(g) + 1e-8)
        clear = np.abs(g) > 0.2 * np.abs(g).max()
        checked += int(clear.sum())
        assert np.allclose(after[name][clear], want[clear], rtol=0, atol=2e-3 * lr), name
        assert np.all(np.abs(after[name] - P[name]) <= lr * (1 + 1e-5) + 1e-7), name
    assert checked > 200


def test_mdn_training_loop_equals_single_steps(torch_dev):
    """cmh_mdn_train (pairs and Adam steps enqueued by the library) gives the
    parameters and last losses of the same steps taken one call at a time."""
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    rows, steps, lr, seed = 1024, 6, 1e-3, 9
    say("[mdn] training loop against single steps")
    a, b = chromh.MDN(seed=4), chromh.MDN(seed=4)
    la = torch.empty(rows, dtype=torch.float32, device="cuda")
    for q in range(steps):
        X, Z = chromh.mdn_pairs(W.SMALL.model, seed, 17 + q * rows, rows)
        a.train_step(X, Z, 3 + q, lr, loss=la)
    buf = (torch.empty((rows, 576), dtype=torch.bfloat16, device="cuda"),
           torch.empty((rows, 3), dtype=torch.float32, device="cuda"))
    lb = torch.empty(rows, dtype=torch.float32, device="cuda")
    b.train(W.SMALL.model, seed, 17, steps, rows, 3, lr, buf, loss=lb)
    torch.cuda.synchronize()
    assert np.array_equal(a.get_params(), b.get_params())
    assert torch.equal(la, lb)
    with pytest.raises(chromh.CmhError):
        b.train(W.PAPER1D.model, seed, 0, 1, rows, 1, lr, buf)   # no training pairs on the line
    with pytest.raises(chromh.CmhError):
        b.train(W.SMALL.model, seed, 0, 0, rows, 1, lr, buf)     # no steps


def test_mdn_pairs_match_oracle(torch_dev):
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    first, count = (1 << 33) + 5, 96     # pair index above 2^32: both counter words used
    say(f"[mdn] pairs first={first} count={count}")
    X, Z = chromh.mdn_pairs(W.SMALL.model, 21, first, count)
    Xg = X.float().cpu().numpy().astype(np.float64)
    Zg = Z.cpu().numpy().astype(np.float64)
    F, T = oracle_pairs(21, first, count)
    assert np.array_equal(Zg, T)
    same = Xg == F
    # binary64 libm results (log, exp, sin, cos) may differ in the last bit
    # between the device and glibc; after rounding to BF16 that shows up only
    # where a value sits on a rounding boundary, as one BF16 ulp
    assert same.mean() > 0.999, same.mean()
    ulp = np.abs(F) * 2.0 ** -7
    assert np.all(np.abs(Xg - F)[~same] <= ulp[~same])


@pytest.mark.parametrize("which", ["small-f64", "dyn10x10-f32"])
def test_anchor_features_match_oracle(torch_dev, which):
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    w = W.SMALL if which == "small-f64" else dynamic_small()
    say(f"[mdn] anchors {w.name}")
    m, _, _, s = instance(w)
    na, ntau = chromh.anchor_count(w.model)
    assert ntau == (w.model.N - 67) // 32 + 1 and na == w.model.nsx * w.model.nsy * ntau
    dt = torch.float64 if w.trace_dtype == "f64" else torch.float32
    trace = torch.from_numpy(np.ascontiguousarray(s)).to(dt).cuda()
    X, wts = chromh.anchor_features(w.model, trace)
    Xg = X.float().cpu().numpy().astype(np.float64)
    wg = wts.cpu().numpy()
    sd = np.asarray(s, dtype=np.float64)
    rng = np.random.default_rng(0)
    picks = np.unique(np.concatenate([[0, na - 1], rng.choice(na, min(na, 120), replace=False)]))
    for a in picks:
        f = D.to_bf16(D.anchor_features(m, sd, ntau, int(a)))
        same = Xg[a] == f
        assert same.mean() > 0.99, a
        assert np.all(np.abs(Xg[a] - f)[~same] <= np.abs(f[~same]) * 2.0 ** -7)
        assert wg[a] == pytest.approx(D.anchor_weight(f), abs=1e-4)


def test_mdn_training_reduces_held_out_loss(torch_dev):
    """Training on simulator pairs lowers the held-out mixture NLL well below
    that of the initial network and of a broad single Gaussian."""
    from paper_1612_00595_amd import chromh
    torch = torch_dev
    say("[mdn] training 300 steps")
    Xtr, Ztr = chromh.mdn_pairs(W.SMALL.model, 5, 0, 16384)
    Xte, Zte = chromh.mdn_pairs(W.SMALL.model, 5, 1 << 20, 2048)
    net = chromh.MDN(seed=3)
    l0, _ = net.gradients(Xte, Zte)
    l0 = float(l0.mean())
    B = 512
    for step in range(1, 301):
        q = ((step - 1) * B) % 16384
        net.train_step(Xtr[q:q + B], Ztr[q:q + B], step, 1e-3)
    l1, _ = net.gradients(Xte, Zte)
    l1 = float(l1.mean())
    torch.cuda.synchronize()
    # targets: x, y uniform on (-1, 1), t / 32 uniform on (-0.5, 2): the
    # log-density of the uniform target box is -ln(2 * 2 * 2.5)
    box = np.log(10.0)
    say(f"[mdn]   held-out NLL {l0:.3f} -> {l1:.3f} (uniform box {box:.3f})")
    assert np.isfinite(l1) and l1 < l0 - 1.0 and l1 < box - 1.0
