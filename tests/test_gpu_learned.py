"""Learned form on the GPU: the start-vector network's kernels against the FP64
oracle (forward, gradients, Adam), and the Galerkin (eq. (5)) and network start
vectors inside the RKC stage loop, where CG to the tolerance stays the judge.

The network's outputs and gradients are compared element by element with the
FP64 oracle in the same operand precision (in BF16 mode the oracle rounds the
operands of every product to bfloat16, as the kernels do), each entry against
its own error scale (the sum of the magnitudes of the terms that form it).
"""

import numpy as np
import pytest

import eqsgen
from oracle import mlp as omlp
from oracle.eqs import EqsOracle

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

from paper_1612_09447_amd import EQS_PREC_FP64, Context, Mlp  # noqa: E402

DEV = torch.device("cuda:0")


def F32(a):
    return torch.as_tensor(np.ascontiguousarray(a, dtype=np.float32), device=DEV)


def params64(p):
    return {k: np.asarray(v, np.float64) for k, v in p.items()}


def abs_forward(p, x, bf16):
    """Magnitude pass of the network: |W| |a| + |b| per layer, with |a| the
    oracle's activations (rounded like the operands in the BF16 form). Each
    output's error scale: a relative perturbation of every operand of the
    sums moves the output by at most that fraction of this value."""
    q = omlp.round_bf16 if bf16 else (lambda v: v)
    y, (xx, h1, a1, h2, a2) = omlp.forward(p, x, bf16)
    A1 = np.abs(q(x)) @ np.abs(q(p["W1"])).T + np.abs(p["b1"])
    A2 = (np.abs(q(a1)) + 1.1 * A1) @ np.abs(q(p["W2"])).T + np.abs(p["b2"])
    A3 = (np.abs(q(a2)) + 1.1 * A2) @ np.abs(q(p["W3"])).T + np.abs(p["b3"])
    return y, A3


def elementwise(got, ref, scale, tol, what):
    """Every |got_i - ref_i| / scale_i <= tol, and all but 1 % of them within
    1e-5 (FP32 rounding of the sums); reported."""
    r = np.abs(np.asarray(got, np.float64) - ref) / np.maximum(scale, 1e-300)
    print(f"[learned] {what}: worst element error {r.max():.2e} of its scale (bar {tol:g}), "
          f"{(r > 1e-5).mean() * 100:.2f} % above 1e-5", flush=True)
    assert r.max() <= tol, (what, r.max(), np.unravel_index(r.argmax(), r.shape))
    assert (r > 1e-5).mean() <= 0.01, what


# Element-wise bars against the oracle in the same operand precision (BF16:
# operands rounded to bfloat16 on both sides): FP32 accumulation of up to 64
# terms through three layers stays within 2e-6 of each output's scale (measured
# worst 2e-7); in BF16
# an operand may round to the neighbouring bfloat16 value on one side only
# (the GPU rounds an FP32 value, the oracle the FP64 one), which moves one term
# by 2^-8 of its size, so the bar is 2^-8 of the scale.
TOL = {False: 2e-6, True: 2.0 ** -8}


@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_forward_matches_oracle(bf16):
    p = eqsgen.mlp_init(4)
    net = Mlp(p, bf16=bf16, stream=torch.cuda.current_stream(DEV))
    rng = np.random.default_rng(0)
    x = rng.normal(size=(100, 32)).astype(np.float32)  # two chunks of <= 64
    y = torch.zeros((100, 16), dtype=torch.float32, device=DEV)
    net.forward(F32(x), y)
    ref, scale = abs_forward(params64(p), x.astype(np.float64), bf16)
    elementwise(y.cpu().numpy(), ref, scale, TOL[bf16], f"forward bf16={bf16}")
    net.close()


def grad_scales(p, x, t, bf16):
    """Per-entry error scale of each gradient: the sum of |terms| of its last
    product (batch sums of |error| x |activation|), plus the propagated
    magnitude of the layer errors."""
    q = omlp.round_bf16 if bf16 else (lambda v: v)
    y, (xx, h1, a1, h2, a2) = omlp.forward(p, x, bf16)
    B, K = y.shape
    dy = np.abs(2.0 * (y - t) / (B * K))
    dh2 = (np.abs(q(dy)) @ np.abs(q(p["W3"]))) * 1.1
    dh1 = (np.abs(q(dh2)) @ np.abs(q(p["W2"]))) * 1.1
    return {"W3": np.abs(q(dy)).T @ np.abs(q(a2)), "b3": dy.sum(0),
            "W2": np.abs(q(dh2)).T @ (np.abs(q(a1)) + 1e-30), "b2": dh2.sum(0),
            "W1": np.abs(q(dh1)).T @ np.abs(q(x)), "b1": dh1.sum(0)}


@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_train_step_gradients_and_adam(bf16):
    p = eqsgen.mlp_init(5)
    net = Mlp(p, bf16=bf16, lr=1e-3, stream=torch.cuda.current_stream(DEV))
    rng = np.random.default_rng(1)
    x = rng.normal(size=(64, 32)).astype(np.float32)
    t = rng.normal(size=(64, 16)).astype(np.float32)
    loss = net.train_step(F32(x), F32(t))
    P64, x64, t64 = params64(p), x.astype(np.float64), t.astype(np.float64)
    L, g = omlp.backward(P64, x64, t64, bf16)
    assert abs(loss - L) <= 1e-5 * L
    p_after, g_gpu = net.get()
    sc = grad_scales(P64, x64, t64, bf16)
    for k in omlp.NAMES:
        elementwise(g_gpu[k], g[k], sc[k], TOL[bf16], f"gradient {k} bf16={bf16}")
    # one Adam step of the oracle from the GPU's own gradients: the FP32 master
    # weights agree to FP32 rounding of the update
    q = params64(p)
    st = omlp.adam_state(q)
    omlp.adam_step(q, params64(g_gpu), st, lr=1e-3)
    for k in omlp.NAMES:
        np.testing.assert_allclose(np.asarray(p_after[k], np.float64), q[k], rtol=0,
                                   atol=2e-7 * (np.abs(q[k]).max() + 1e-3))  # ~2 FP32 ulps
    net.close()


@pytest.mark.parametrize("bf16", [False, True])
def test_mlp_learns_a_linear_map(bf16):
    p = eqsgen.mlp_init(6)
    net = Mlp(p, bf16=bf16, lr=1e-3, stream=torch.cuda.current_stream(DEV))
    rng = np.random.default_rng(2)
    A = rng.normal(size=(16, 32)) / 6
    X = rng.normal(size=(512, 32)).astype(np.float32)
    Y = (X @ A.T).astype(np.float32)
    Xd, Yd = F32(X), F32(Y)
    first = net.train_step(Xd[:64], Yd[:64])
    for it in range(1, 400):
        b = rng.choice(512, 64, replace=False)
        last = net.train_step(Xd[b], Yd[b])
    assert last < 0.05 * first, (first, last)
    net.close()


def run_kind(case, kind, steps, rtol, **kw):
    o = EqsOracle(case)
    with Context(0, torch.cuda.current_stream(DEV)) as c:
        c.setup_case(case, precision=EQS_PREC_FP64)
        if kind == "mlp":
            c.set_guess("mlp", init=eqsgen.mlp_init(4), **kw)
        else:
            c.set_guess(kind, **kw)
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        traj, stats = [], []
        for n in range(steps):
            st = c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=rtol, maxit=500, allow_not_converged=True)
            if st["not_converged"]:
                print(f"[guess] {kind} step {n}: {st}", flush=True)
            assert st["not_converged"] == 0, (kind, n, st)
            stats.append(st)
            traj.append(x.cpu().numpy()[o.free].copy())
    return traj, stats, o


def test_start_vector_kinds_keep_the_result_and_galerkin_beats_previous():
    case = eqsgen.case_c1(n=12, seed=1)
    case.s = 12
    steps = 8
    o = EqsOracle(case)
    ref = o.rkc_trajectory(np.zeros(o.n_free), 0.0, case.tau, case.s, steps)[1:]
    scale = max(np.linalg.norm(r) for r in ref)
    iters = {}
    runs = [("previous", "previous", {}), ("zero", "zero", {}), ("galerkin", "galerkin", {}),
            ("mlp", "mlp", dict(warmup=16)),
            # the paper's other estimators: a fixed POD basis (MOR) and a sliding
            # window that takes only solutions whose solve exceeded an iteration
            # count (MOR2)
            ("mor", "mor", dict(window=8)), ("mor2", "galerkin", dict(add_threshold=8))]
    for label, kind, kw in runs:
        traj, stats, _ = run_kind(case, kind, steps, 1e-11, **kw)
        err = max(np.linalg.norm(a - b) for a, b in zip(traj, ref)) / scale
        iters[label] = sum(s["total_iters"] for s in stats)
        used = sum(s["guess_used"] for s in stats)
        fb = sum(s["guess_fallbacks"] for s in stats)
        print(f"[guess] {label}: CG iterations {iters[label]}, used {used}, fallbacks {fb}, err {err:.2e}, "
              f"loss {stats[-1]['train_loss']:.3e}", flush=True)
        assert err <= 1e-9, (label, err)
        if kind != "previous" and kind != "zero":
            assert used + fb > 0, label
    assert iters["galerkin"] < iters["previous"] < iters["zero"]
    assert iters["mlp"] < iters["previous"]  # what the trained network gains over the plain method
    assert iters["mor"] < iters["zero"] and iters["mor2"] < iters["zero"]


def test_galerkin_start_vector_matches_oracle():
    """Eq. (5) through eqs_galerkin_start (the coefficient solve of a stage's
    Galerkin start vector) against the oracle's POD basis and reduced solve, on
    windows of seeded vectors: full rank (every direction kept), one exactly
    dependent column (one direction dropped) and a single column (closed form
    s (s^T r) / (s^T M s)); Galerkin orthogonality S^T (r - M x0) = 0 holds."""
    from oracle.guess import galerkin_start, pod_from_gram

    from paper_1612_09447_amd import EqsError

    case = eqsgen.case_c1(n=12, seed=1)
    o = EqsOracle(case)
    nf = o.n_free
    rng = np.random.default_rng(11)
    base = rng.standard_normal((nf, 6))
    windows = {
        "full": base,
        "dependent": np.column_stack([base[:, :4], base[:, 0] + 2.0 * base[:, 2], base[:, 4]]),
        "single": base[:, :1],
    }
    r = rng.standard_normal(nf)
    with Context(0, torch.cuda.current_stream(DEV)) as c:
        c.setup_case(case, precision=EQS_PREC_FP64)
        rd = torch.from_numpy(r).to(DEV)
        for label, S in windows.items():
            k = S.shape[1]
            R = o.M_II @ S
            Sd = torch.from_numpy(np.ascontiguousarray(S.T)).to(DEV)
            Rd = torch.from_numpy(np.ascontiguousarray(R.T)).to(DEV)
            x0 = torch.full((nf,), float("nan"), dtype=torch.float64, device=DEV)
            m = c.galerkin_start(Sd, Rd, rd, x0)
            got = x0.cpu().numpy()
            V, sig, _ = pod_from_gram(S, 16)
            want = galerkin_start(V, o.M_II, r)
            err = np.linalg.norm(got - want) / np.linalg.norm(want)
            orth = np.linalg.norm(S.T @ (r - o.M_II @ got)) / (np.linalg.norm(S, axis=0).max() * np.linalg.norm(r))
            print(f"[galerkin] {label}: k {k}, kept {m} (oracle {V.shape[1]}), rel err {err:.2e}, "
                  f"orthogonality {orth:.2e}", flush=True)
            assert m == V.shape[1] == {"full": 6, "dependent": 5, "single": 1}[label]
            assert err <= 1e-10, (label, err)
            assert orth <= 1e-11, (label, orth)
            if label == "single":
                s = S[:, 0]
                closed = s * (s @ r) / (s @ (o.M_II @ s))
                assert np.linalg.norm(got - closed) <= 1e-12 * np.linalg.norm(closed)
        # x0 over its own window is refused before any launch
        with pytest.raises(EqsError):
            c.galerkin_start(Sd, Rd, rd, Sd[0])


def test_setting_the_start_vector_again_keeps_device_memory():
    """eqs_set_guess on a context that already ran guessed stages replaces the
    window buffers instead of adding new ones (device_bytes stays put)."""
    case = eqsgen.case_c1(n=10, seed=1)
    case.s = 8
    with Context(0, torch.cuda.current_stream(DEV)) as c:
        c.setup_case(case, precision=EQS_PREC_FP64)
        x = torch.zeros(case.n_nodes, dtype=torch.float64, device=DEV)
        sizes = []
        for n, kind in enumerate(["galerkin", "mor", "galerkin"]):
            c.set_guess(kind)
            c.rkc_step(n * case.tau, case.tau, case.s, x, rtol=1e-10, maxit=500)
            sizes.append(c.info()["device_bytes"])
        print(f"[guess] device bytes after each setting: {sizes}", flush=True)
        assert sizes[0] == sizes[1] == sizes[2]
