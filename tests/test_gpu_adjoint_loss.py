"""GPU adjoint, autograd and spectral loss vs the FP64 oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_1507_02525_amd import workloads
from tests.gpu_util import FWD_TOL, GRAD_TOL, log, need_gpu, rel_l2, to_dev

pytestmark = pytest.mark.gpu


def _api():
    import paper_1507_02525_amd.api as api
    return api


@pytest.mark.parametrize("m", [1, 2, 4, 5, 8, 12, 13, 15, 17, 18])
@pytest.mark.parametrize("real", [False, True])
def test_adjoint_vs_oracle(m, real):
    need_gpu()
    log("adjoint m=%d real=%s" % (m, real))
    rng = np.random.default_rng(2000 + m)
    b = 2
    gy = workloads.gaussian_complex(rng, (b, m, 1 << m))
    gx = _api().adjoint(to_dev(gy), real=real).cpu().numpy()
    for s in range(b):
        ref = oracle.adjoint(gy[s].astype(np.complex128))
        if real:
            ref = ref.real
        e = rel_l2(gx[s], ref)
        assert e <= GRAD_TOL, e


def test_adjoint_identity_full_size():
    """Re<A x, g> = Re<x, A^H g> on the benchmark shape (64 x 2^16, real)."""
    need_gpu()
    api = _api()
    d = workloads.make(2)
    x = to_dev(d["x"])
    rng = np.random.default_rng(5)
    g = to_dev(workloads.gaussian_complex(rng, (64, 16, 1 << 16)))
    Y = api.forward(x)
    gx = api.adjoint(g, real=True)
    lhs = torch.sum((torch.conj(g) * Y).to(torch.complex128)).real.item()
    rhs = torch.sum(gx.double() * x.double()).item()
    assert abs(lhs - rhs) <= 1e-5 * abs(lhs)


def test_adjoint_of_forward_is_scaled_identity():
    need_gpu()
    api = _api()
    m = 14
    rng = np.random.default_rng(6)
    x = to_dev(workloads.gaussian_complex(rng, (2, 1 << m)))
    g = api.adjoint(api.forward(x))
    assert rel_l2(g.cpu().numpy(), (2 ** (m + 1) - 2) * x.cpu().numpy()) <= GRAD_TOL


@pytest.mark.parametrize("dtype", [torch.complex64, torch.float32])
def test_autograd_matches_oracle_adjoint(dtype):
    need_gpu()
    api = _api()
    m = 13
    rng = np.random.default_rng(7)
    if dtype == torch.complex64:
        xn = workloads.gaussian_complex(rng, (2, 1 << m))
    else:
        xn = workloads.gaussian_real(rng, (2, 1 << m))
    W = workloads.gaussian_complex(rng, (2, m, 1 << m))
    x = to_dev(xn).requires_grad_(True)
    Y = api.mrdft(x)
    loss = torch.sum((torch.conj(to_dev(W)) * Y).real)
    loss.backward()
    g = x.grad.cpu().numpy()
    for s in range(2):
        ref = oracle.adjoint(W[s].astype(np.complex128))
        if dtype == torch.float32:
            ref = ref.real
        assert rel_l2(g[s], ref) <= GRAD_TOL


def _loss_case(batch, m, seed):
    rng = np.random.default_rng(seed)
    return workloads.gaussian_real(rng, (batch, 1 << m)), workloads.gaussian_real(rng, (batch, 1 << m))


@pytest.mark.parametrize("m", [3, 10, 12, 14, 16, 17])
def test_spectral_loss_vs_oracle(m):
    need_gpu()
    api = _api()
    x, z = _loss_case(3, m, 300 + m)
    num_den, L = api.spectral_loss_terms(to_dev(x), to_dev(z))
    nd = num_den.cpu().numpy()
    Lref = 0.0
    for b in range(3):
        ndr, lr = oracle.spectral_loss(x[b], z[b])
        assert np.max(np.abs(nd[b] / ndr - 1)) <= FWD_TOL
        Lref += lr
    assert abs(L.item() / Lref - 1) <= 1e-6


def test_spectral_loss_gradient_vs_oracle_and_fd():
    need_gpu()
    api = _api()
    m = 6
    x, z = _loss_case(2, m, 99)
    xt = to_dev(x).requires_grad_(True)
    L = api.spectral_loss(xt, to_dev(z))
    (0.75 * L).backward()
    g = xt.grad.cpu().numpy()
    for b in range(2):
        nd, _ = oracle.spectral_loss(x[b], z[b])
        ref = oracle.spectral_loss_grad(x[b], z[b], nd, gL=0.75)
        assert rel_l2(g[b], ref) <= GRAD_TOL
        # FP64 central differences of the oracle loss (exact for a quadratic)
        h = 1e-4
        xd = x[b].astype(np.float64)
        fd = np.empty(1 << m)
        for p in range(1 << m):
            e = np.zeros(1 << m)
            e[p] = h
            fd[p] = 0.75 * (oracle.spectral_loss(xd + e, z[b])[1] - oracle.spectral_loss(xd - e, z[b])[1]) / (2 * h)
        assert rel_l2(g[b], fd) <= GRAD_TOL


@pytest.mark.parametrize("m", [12, 13, 16])
def test_spectral_loss_gradient_fused_orders(m):
    """Gradient through the one-launch path (levels up to 16 recomputed with
    their factors folded in) against the oracle's adjoint-based gradient."""
    need_gpu()
    api = _api()
    x, z = _loss_case(2, m, 500 + m)
    log("loss gradient m=%d" % m)
    xt = to_dev(x).requires_grad_(True)
    L = api.spectral_loss(xt, to_dev(z))
    (1.5 * L).backward()
    g = xt.grad.cpu().numpy()
    for b in range(2):
        nd, _ = oracle.spectral_loss(x[b], z[b])
        ref = oracle.spectral_loss_grad(x[b], z[b], nd, gL=1.5)
        assert rel_l2(g[b], ref) <= GRAD_TOL


def test_workload5_full_size():
    """32 x 2^18 real pairs: loss terms vs the oracle for sampled signals,
    gradient vs the oracle gradient and the closed form 2(x - z)/||z||^2."""
    need_gpu()
    api = _api()
    d = workloads.make(5)
    x, z = d["x"], d["z"]
    log("workload 5 full: 32 x r32 m=18")
    xt = to_dev(x).requires_grad_(True)
    L = api.spectral_loss(xt, to_dev(z))
    L.backward()
    g = xt.grad.cpu().numpy()
    num_den, _ = api.spectral_loss_terms(to_dev(x), to_dev(z))
    nd = num_den.cpu().numpy()
    Lsum = 0.0
    for b in range(32):
        xd = x[b].astype(np.float64)
        zd = z[b].astype(np.float64)
        closed = 2 * (xd - zd) / np.sum(zd ** 2)
        assert rel_l2(g[b], closed) <= GRAD_TOL
        Lsum += np.sum((xd - zd) ** 2) / np.sum(zd ** 2)
    for b in (0, 31):
        ndr, _ = oracle.spectral_loss(x[b], z[b])
        assert np.max(np.abs(nd[b] / ndr - 1)) <= FWD_TOL
        ref = oracle.spectral_loss_grad(x[b], z[b], ndr)
        assert rel_l2(g[b], ref) <= GRAD_TOL
    assert abs(L.item() / Lsum - 1) <= FWD_TOL


@pytest.mark.parametrize("m", [13, 18])
def test_spectral_loss_fwd_graph_replay(m):
    """The loss forward captured into a HIP graph (it clears its sums with a
    fill kernel, no memset node) gives the eager result on every replay, with
    eager work on the stream between the replays."""
    need_gpu()
    api = _api()
    x, z = _loss_case(3, m, 900 + m)
    log("loss forward graph m=%d" % m)
    xd, zd = to_dev(x), to_dev(z)
    plan = api.Plan(m=m, batch=3, dtype="r32")
    nd = torch.empty(3, m, 2, dtype=torch.float64, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    plan.mrdft_spectral_loss_fwd(xd, zd, nd, L)            # eager (allocates the workspace)
    torch.cuda.synchronize()
    nd0, L0 = nd.clone(), L.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.mrdft_spectral_loss_fwd(xd, zd, nd, L)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for r in range(3):
        nd.fill_(-1.0)
        L.fill_(-1.0)
        junk.add_(float(r))                                  # eager work between the replays
        g.replay()
        torch.cuda.synchronize()
        assert torch.allclose(nd, nd0, rtol=1e-12, atol=0.0), r
        assert torch.allclose(L, L0, rtol=1e-6, atol=0.0), r


@pytest.mark.parametrize("m", [13, 18])
def test_spectral_loss_bwd_graph_replay(m):
    """The loss backward captured into a HIP graph: at m = 18 the passes of
    levels 17 and 18 and the heads of the adjoint's pass chains fork onto side
    streams and join back inside the capture.  Every replay, with eager work
    between, gives the eager gradient."""
    need_gpu()
    api = _api()
    x, z = _loss_case(3, m, 950 + m)
    log("loss backward graph m=%d" % m)
    xd, zd = to_dev(x), to_dev(z)
    plan = api.Plan(m=m, batch=3, dtype="r32")
    nd = torch.empty(3, m, 2, dtype=torch.float64, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    gL = torch.full((1,), 0.75, dtype=torch.float32, device="cuda")
    gx = torch.empty(3, 1 << m, dtype=torch.float32, device="cuda")
    plan.mrdft_spectral_loss_fwd(xd, zd, nd, L)
    plan.mrdft_spectral_loss_bwd(xd, zd, nd, gL, gx)        # eager
    torch.cuda.synchronize()
    g0 = gx.clone()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    g = torch.cuda.CUDAGraph()
    with torch.cuda.stream(s):
        with torch.cuda.graph(g, stream=s):
            plan.mrdft_spectral_loss_bwd(xd, zd, nd, gL, gx)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    junk = torch.zeros(1 << 20, device="cuda")
    for r in range(3):
        gx.fill_(-1.0)
        junk.add_(float(r))                                  # eager work between the replays
        g.replay()
        torch.cuda.synchronize()
        assert rel_l2(gx.cpu().numpy().astype(np.float64), g0.cpu().numpy().astype(np.float64)) <= 1e-6, r
    # and the eager gradient itself against the oracle on one signal
    ref = oracle.spectral_loss_grad(x[1], z[1], oracle.spectral_loss(x[1], z[1])[0], gL=0.75)
    assert rel_l2(g0[1].cpu().numpy().astype(np.float64), ref) <= GRAD_TOL


def test_loss_entry_points_check_buffers():
    """The plan's loss calls reject buffers of the wrong size, dtype or plan
    kind before the library is called; a valid call after them still works."""
    need_gpu()
    api = _api()
    m, b = 12, 2
    x, z = _loss_case(b, m, 77)
    xd, zd = to_dev(x), to_dev(z)
    plan = api.Plan(m=m, batch=b, dtype="r32")
    nd = torch.empty(b, m, 2, dtype=torch.float64, device="cuda")
    L = torch.empty(1, dtype=torch.float32, device="cuda")
    gL = torch.ones(1, dtype=torch.float32, device="cuda")
    gx = torch.empty(b, 1 << m, dtype=torch.float32, device="cuda")
    with pytest.raises(ValueError):
        plan.mrdft_spectral_loss_fwd(xd, zd[:1], nd, L)                    # z of one signal
    with pytest.raises(ValueError):
        plan.mrdft_spectral_loss_fwd(xd, zd, nd[:1], L)                    # num_den too short
    with pytest.raises(ValueError):
        plan.mrdft_spectral_loss_fwd(xd, zd, nd.float(), L)                # num_den not float64
    with pytest.raises(ValueError):
        plan.mrdft_spectral_loss_bwd(xd, zd, nd, gL, gx[:1])               # gx too short
    with pytest.raises(ValueError):
        api.Plan(m=m, batch=b, dtype="c64").mrdft_spectral_loss_fwd(xd, zd, nd, L)
    plan.mrdft_spectral_loss_fwd(xd, zd, nd, L)
    plan.mrdft_spectral_loss_bwd(xd, zd, nd, gL, gx)
    torch.cuda.synchronize()
    ref = oracle.spectral_loss_grad(x[1], z[1], oracle.spectral_loss(x[1], z[1])[0])
    assert rel_l2(gx[1].cpu().numpy().astype(np.float64), ref) <= GRAD_TOL
