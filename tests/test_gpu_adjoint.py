"""GPU parity of the adjoint (edge-weight gradient of the summed scores) against the FP64 oracle.

Gradient of L = <g, S~> (log-scale fixed) per stored entry: e^{-Sigma} G_ij with
G = int_0^1 e^{sA} g 1^T e^{(1-s)A} ds. Checked against the dense Van Loan block exponential
(FP64 mode: 1e-9 normwise), dense Van Loan at n=500 in FP32 (1e-4 normwise), central differences of
the FP64 oracle Lanczos on sampled undirected edges (h = 1e-3; per edge |grad - fd| <= 1e-6 |fd| +
1e-9 max|grad| in FP64 mode, 1e-5 |fd| + 1e-6 max|grad| in FP32), the Euler identity, and autograd.
"""
import numpy as np
import pytest
import scipy.sparse as sp

from fixtures import configs as C
from oracle import dense as odense, gradient as ograd, lanczos as olanczos
from tests import graphs_small as gs
from tests.test_gpu_parity import DenseBatch

pytestmark = pytest.mark.gpu


def api():
    from paper_1409_5000_amd import api as _api
    return _api


def torch_mod():
    import torch
    return torch


def dense_reference(hb, b, g_blocks, log_scale):
    """Per-entry reference gradient e^{-Sigma} G_ij from the dense Van Loan route (shifted by lambda_max)."""
    ref = np.empty(int(hb.nnz_off[-1]))
    for r in range(hb.R):
        n, rp, ci, v = hb.csr(r)
        A = odense.csr_to_scipy(n, rp, ci, v).toarray()
        gi = int(hb.graph_of[r])
        th = float(np.linalg.eigvalsh(A)[-1])
        G = ograd.grad_vanloan(A - th * np.eye(n), g_blocks[gi]) * np.exp(th - log_scale[gi])
        rows = np.repeat(np.arange(n), np.diff(rp))
        ref[hb.nnz_off[r]:hb.nnz_off[r + 1]] = G[rows, ci]
    return ref


def weighted_dense_batch(graphs, dtype, seed=0):
    hb = DenseBatch(graphs, dtype, weighted=True)
    rng = np.random.default_rng(seed)
    vals = np.empty(hb.col_idx.size)
    for r in range(hb.R):   # symmetric weights in (0.5, 1.5)
        n, rp, ci, _ = hb.csr(r)
        rows = np.repeat(np.arange(n), np.diff(rp))
        W = np.triu(rng.uniform(0.5, 1.5, (n, n)), 1)
        W = W + W.T
        vals[hb.nnz_off[r]:hb.nnz_off[r + 1]] = W[rows, ci]
    hb.values = vals.astype(hb.dtype)
    return hb


@pytest.mark.parametrize("n,p,m", [(7, 0.6, 8), (15, 0.4, 16), (22, 0.3, 24)])
def test_adjoint_fp64_small_dimensions_exact(gpu_lib, n, p, m):
    # m >= n: both Krylov spaces are the whole space (Lanczos stops at breakdown), so the gradient is
    # the exact one; covers the 8-, 16- and 24-column forms of the Z build and the SDDMM
    torch = torch_mod()
    graphs = [[gs.random_graph(n, p, 11 + n), gs.random_graph(n, p, 12 + n)], [gs.random_graph(n, p, 13 + n)]]
    hb = weighted_dense_batch(graphs, "f64", seed=n)
    b = api().Batch.from_host(hb)
    out = b.scores(m=m)
    rng = np.random.default_rng(n)
    g_blocks = [rng.normal(size=int(k)) for k in hb.n]
    gt = torch.as_tensor(np.concatenate(g_blocks)).to("cuda")
    grad = b.scores_backward(out.log_scale, gt, m=m)
    torch.cuda.synchronize()
    ref = dense_reference(hb, b, g_blocks, out.log_scale.cpu().numpy())
    got = grad.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_adjoint_fp64_vs_dense_vanloan(gpu_lib):
    torch = torch_mod()
    graphs = [[gs.random_graph(120, 0.08, 1), gs.random_graph(120, 0.1, 2)], [gs.random_graph(90, 0.12, 3)]]
    hb = weighted_dense_batch(graphs, "f64", seed=4)
    b = api().Batch.from_host(hb)
    out = b.scores(m=40)
    rng = np.random.default_rng(7)
    g_blocks = [rng.normal(size=int(n)) for n in hb.n]
    gt = torch.as_tensor(np.concatenate(g_blocks)).to("cuda")
    grad = b.scores_backward(out.log_scale, gt, m=40)
    torch.cuda.synchronize()
    ref = dense_reference(hb, b, g_blocks, out.log_scale.cpu().numpy())
    got = grad.cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref))


def test_adjoint_fp32_n500_vs_dense(gpu_lib):
    # a fresh instance of the differentiation recipe at n=500 (degree 16, 40-node target, m=30)
    torch = torch_mod()
    w = C.scaled(C.workload(3), n=500, N=2)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    out = b.scores(m=w.m)
    g = np.zeros(500)
    g[b_targets(hb)] = 1.0   # loss = sum of the summed scores over the target nodes
    grad = b.scores_backward(out.log_scale, torch.as_tensor(g).to("cuda"), m=w.m)
    torch.cuda.synchronize()
    ref = dense_reference(hb, b, [g], out.log_scale.cpu().numpy())
    got = grad.double().cpu().numpy()
    assert np.max(np.abs(got - ref)) <= 1e-4 * np.max(np.abs(ref))


def b_targets(hb, gi=0):
    return np.asarray(hb.targets[gi], dtype=np.int64)


_FD_SHARED = {}  # the batch and cotangent, inherited by the forked workers instead of pickled per job


def _fd_job(args):
    # central difference of the loss in the weight of one undirected edge: entries e = (i, j) and
    # e2 = (j, i) of realization r move together
    r, e, e2, h, sigma, m = args
    hb, gvec = _FD_SHARED["hb"], _FD_SHARED["g"]
    n, rp, ci, v = hb.csr(r)
    base = odense.csr_to_scipy(n, rp, ci, v)
    vals = []
    for sgn in (1.0, -1.0):
        B = base.copy()
        B.data[e] += sgn * h
        B.data[e2] += sgn * h
        res = olanczos.lanczos_expv(B, m=m)
        vals.append(np.exp(res.theta - sigma) * float(gvec @ res.u))
    return (vals[0] - vals[1]) / (2 * h)


def fd_check(hb, b, out, grad, m, nedges, seed, tol_rel, tol_abs_frac, workers=8):
    import multiprocessing as mp
    rng = np.random.default_rng(seed)
    sigma = float(out.log_scale.cpu().numpy()[0])
    g = np.zeros(int(hb.n[0]))
    g[b_targets(hb)] = 1.0
    jobs, gpu_vals = [], []
    gpu = grad.double().cpu().numpy()
    for _ in range(nedges):
        r = int(rng.integers(0, hb.R))
        n, rp, ci, _ = hb.csr(r)
        e = int(rng.integers(0, ci.size))
        i = int(np.searchsorted(rp, e, side="right") - 1)
        j = int(ci[e])
        # entry (j, i) of the same realization
        e2 = int(rp[j] + np.searchsorted(ci[rp[j]:rp[j + 1]], i))
        gpu_vals.append(gpu[hb.nnz_off[r] + e] + gpu[hb.nnz_off[r] + e2])
        jobs.append((r, e, e2, 1e-3, sigma, m))
    _FD_SHARED.update(hb=hb, g=g)
    try:
        with mp.get_context("fork").Pool(workers) as pool:
            fd = np.array(pool.map(_fd_job, jobs))
    finally:
        _FD_SHARED.clear()
    gpu_vals = np.array(gpu_vals)
    scale = np.max(np.abs(gpu))
    err = np.abs(gpu_vals - fd)
    big = np.abs(fd) > 1e-3 * scale
    print(f"fd check: {nedges} edges, max|grad| {scale:.3e}, worst |err|/|fd| on edges with |fd| > 1e-3 max|grad| "
          f"{np.max(err[big] / np.abs(fd[big])) if big.any() else 0.0:.3e}, worst |err|/max|grad| {err.max() / scale:.3e}")
    assert np.all(err <= tol_rel * np.abs(fd) + tol_abs_frac * scale), (err.max(), np.abs(fd).max(), scale)


def test_adjoint_fp32_central_differences_reduced(gpu_lib):
    torch = torch_mod()
    w = C.scaled(C.workload(3), n=20000, N=4)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    out = b.scores(m=w.m)
    g = np.zeros(int(hb.n[0]))
    g[b_targets(hb)] = 1.0
    grad = b.scores_backward(out.log_scale, torch.as_tensor(g).to("cuda"), m=w.m)
    torch.cuda.synchronize()
    fd_check(hb, b, out, grad, w.m, nedges=24, seed=3, tol_rel=1e-5, tol_abs_frac=1e-6)


def test_adjoint_fp64_central_differences_multiblock(gpu_lib):
    # FP64 mode with several 2048-row blocks per realization (the cross-block dot and norm partials,
    # the Z build and the SDDMM across blocks): the differentiation recipe at n = 12000 (six row
    # blocks), three realizations, symmetric weights in [0.5, 1.5), m = 30; 100 random edges against
    # central differences of the FP64 oracle Lanczos with h = 1e-3, per edge
    # |grad - fd| <= 1e-6 |fd| + 1e-9 max|grad| (the difference quotient's own truncation at this h is
    # below 3e-7 relative: it moves by 2.4e-7 between h = 1e-3 and 5e-4)
    import dataclasses
    torch = torch_mod()
    w = dataclasses.replace(C.scaled(C.workload(3), n=12000, N=3), dtype="f64")
    hb = C.build(w)
    vals = np.empty(hb.col_idx.size)
    for r in range(hb.R):
        n, rp, ci, _ = hb.csr(r)
        rows = np.repeat(np.arange(n), np.diff(rp))
        lo, hi = np.minimum(rows, ci), np.maximum(rows, ci)
        h = (lo.astype(np.int64) * 2654435761 + hi * 40503 + r * 977) % 1000
        vals[hb.nnz_off[r]:hb.nnz_off[r + 1]] = 0.5 + h / 1000.0
    hb.values = vals
    b = api().Batch.from_host(hb)
    out = b.scores(m=w.m)
    g = np.zeros(int(hb.n[0]))
    g[b_targets(hb)] = 1.0
    grad = b.scores_backward(out.log_scale, torch.as_tensor(g).to("cuda"), m=w.m)
    torch.cuda.synchronize()
    assert grad.dtype == torch.float64
    fd_check(hb, b, out, grad, w.m, nedges=100, seed=17, tol_rel=1e-6, tol_abs_frac=1e-9, workers=16)


def test_adjoint_euler_identity_fp32(gpu_lib):
    # sum_e A_e grad_e = sum_k e^{theta_k - Sigma} g^T A_k u_k (d/dt <g, S~(tA)> at t = 1)
    torch = torch_mod()
    w = C.scaled(C.workload(3), n=30000, N=3)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    out = b.scores(m=w.m)
    g = np.random.default_rng(1).normal(size=int(hb.n[0]))
    grad = b.scores_backward(out.log_scale, torch.as_tensor(g).to("cuda"), m=w.m)
    torch.cuda.synchronize()
    sigma = float(out.log_scale.cpu().numpy()[0])
    lhs = float(np.dot(hb.values.astype(np.float64), grad.double().cpu().numpy()))
    rhs = 0.0
    for r in range(hb.R):
        n, rp, ci, v = hb.csr(r)
        A = odense.csr_to_scipy(n, rp, ci, v)
        res = olanczos.lanczos_expv(A, m=w.m)
        rhs += np.exp(res.theta - sigma) * float(g @ (A @ res.u))
    assert abs(lhs - rhs) <= 1e-5 * abs(rhs)


def test_autograd_function_matches_backward(gpu_lib):
    torch = torch_mod()
    w = C.scaled(C.workload(3), n=5000, N=2)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    values = b.values
    values.requires_grad_(True)
    scores, log_scale = api().Communicability.apply(values, b, {"m": w.m})
    loss = scores[torch.as_tensor(b_targets(hb)).to("cuda")].sum()
    loss.backward()
    g = torch.zeros(int(hb.n[0]), dtype=torch.float32, device="cuda")
    g[torch.as_tensor(b_targets(hb)).to("cuda")] = 1.0
    direct = b.scores_backward(log_scale, g, m=w.m)
    torch.cuda.synchronize()
    assert torch.equal(values.grad, direct)


def test_backward_checks_the_forward_checkpoint(gpu_lib):
    # the forward call's checkpoint (alpha, beta, theta*, beta0, steps, flags) against the backward's
    # recomputed forward: equal bit for bit, so the count is 0 and the gradient is the unchecked one;
    # a changed checkpoint entry is counted; weights changed in place between the autograd forward
    # and backward make the backward raise
    torch = torch_mod()
    w = C.scaled(C.workload(3), n=3000, N=3)
    hb = C.build(w)
    b = api().Batch.from_host(hb)
    out = b.scores(m=w.m, ckpt=True)
    g = torch.zeros(int(hb.n[0]), dtype=torch.float32, device="cuda")
    g[torch.as_tensor(b_targets(hb)).to("cuda")] = 1.0
    plain = b.scores_backward(out.log_scale, g, m=w.m).clone()
    bwd = b.backward_run(m=w.m)
    grad, mism = bwd.launch(out.log_scale, g, out.ckpt)
    torch.cuda.synchronize()
    assert int(mism.item()) == 0 and torch.equal(grad, plain)
    bad = out.ckpt.clone()
    bad.view(3, -1)[1, 0] = torch.nextafter(bad.view(3, -1)[1, 0], torch.tensor(1e300, dtype=torch.float64, device="cuda"))
    _, mism = bwd.launch(out.log_scale, g, bad)
    torch.cuda.synchronize()
    assert int(mism.item()) == 1
    with pytest.raises(RuntimeError, match="differs from the forward checkpoint"):
        b.scores_backward(out.log_scale, g, ckpt=bad, m=w.m)
    values = b.values
    values.requires_grad_(True)
    scores, _ = api().Communicability.apply(values, b, {"m": w.m})
    with torch.no_grad():
        values[0] *= 1.5  # the weights the backward would recompute with are no longer the forward's
    with pytest.raises(RuntimeError, match="differs from the forward checkpoint"):
        scores[torch.as_tensor(b_targets(hb)).to("cuda")].sum().backward()


def test_zero_cotangent_gives_zero_gradient(gpu_lib):
    torch = torch_mod()
    hb = weighted_dense_batch([[gs.random_graph(100, 0.1, 5)]], "f64")
    b = api().Batch.from_host(hb)
    out = b.scores(m=20)
    grad = b.scores_backward(out.log_scale, torch.zeros(100, dtype=torch.float64, device="cuda"), m=20)
    torch.cuda.synchronize()
    assert torch.count_nonzero(grad).item() == 0


def test_adjoint_full_size_central_differences(gpu_lib):
    # the differentiation workload at full size: ER n=2e5 degree 16, 16 realizations, m=30, FP32
    # weights at 1.0; loss = sum of the summed scores over the 40 target nodes; 100 random edges
    torch = torch_mod()
    w = C.workload(3)
    hb = C.build_parallel(w, workers=16)
    b = api().Batch.from_host(hb)
    out = b.scores(m=w.m)
    g = np.zeros(int(hb.n[0]))
    g[b_targets(hb)] = 1.0
    grad = b.scores_backward(out.log_scale, torch.as_tensor(g).to("cuda"), m=w.m)
    torch.cuda.synchronize()
    fd_check(hb, b, out, grad, w.m, nedges=100, seed=11, tol_rel=1e-5, tol_abs_frac=1e-6, workers=16)
