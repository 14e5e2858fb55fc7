"""GPU path-replay adjoint vs the oracle's gradient estimator, closed-form
derivatives and central finite differences with common random numbers."""
from __future__ import annotations

import math

import numpy as np
import pytest

import closed_forms as cf
import oracle
import workloads
from replay import check_grad_total, compare_records, oracle_replay
from stats import check_z

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    torch.cuda.set_device(0)
    yield
    torch.cuda.synchronize()


def _fpt():
    import paper_1706_03024_amd as fpt
    return fpt


def _gfilm(scene, seed=3):
    rng = np.random.default_rng(seed)
    return 1.0 + rng.random(oracle.film_shape(scene))


def test_adjoint_per_path_replay_and_total():
    """Same random streams: each path's gradient contribution matches the
    oracle's (fp32 vs fp64, relative 1e-5 scaled by the path's condition
    number), and fpt_render_adjoint's total equals the sum of the per-path
    contributions and the oracle's total."""
    import torch
    fpt = _fpt()
    scene = workloads.cornell_scene(24, 24)
    for m in range(3):  # brighter dyes so every parameter matters
        scene["media"][m]["dyes"][0][1] *= 20
    run = workloads.make_run(1 << 15, seed=8)
    g = _gfilm(scene)
    sc = fpt.Scene(scene)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    rec, rg = sc.records(run, grad_film=gt)
    total = sc.render_adjoint(run, gt)
    torch.cuda.synchronize()
    total = total.cpu().numpy().astype(np.float64)
    sc.close()
    cond = oracle_replay(scene, run, grad_film=g)
    print(compare_records(rec, cond, gpu_grad=rg))
    print("total deviations", check_grad_total(total, rg, cond))


def test_adjoint_dye_slab_closed_form():
    """Non-scattering dye slab: GPU gradient of the total fluorescent escape
    w.r.t. concentration and QY equals the closed-form derivative."""
    import torch
    fpt = _fpt()
    conc, qy = 20.0, 0.8
    scene = workloads.t6_dye_slab(conc_uM=conc, qy=qy)
    N = 101

    def fl_total(c, q):
        lam = cf.grid_lambda(N)
        sa = cf.dye_sigma_a(lam, [(490, 20, 1)], 7e4, c, N)
        st = 0.05 + sa
        R, T = cf.dye_slab_fluorescent_film(1.0, st[38], sa[38], q, cf.emission_pmf(N, [(520, 25, 1)]), st)
        return R.sum() + T.sum()

    h = 1e-4
    d_c = (fl_total(conc * (1 + h), qy) - fl_total(conc * (1 - h), qy)) / (2 * h * conc)
    d_q = (fl_total(conc, qy * (1 + h)) - fl_total(conc, qy * (1 - h))) / (2 * h * qy)
    sc = fpt.Scene(scene)
    g = torch.zeros(sc.film_shape(), device="cuda")
    g[0, 1] = 1.0
    B, n = 32, 1 << 18
    est = []
    for b in range(B):
        est.append(sc.render_adjoint(workloads.make_run(n, seed=100 + b), g).cpu().numpy())
    sc.close()
    est = np.array(est, dtype=np.float64)
    m, se = est.mean(0), est.std(0, ddof=1) / math.sqrt(B)
    check_z([(m[0] - d_c) / se[0], (m[1] - d_q) / se[1]], "GPU dye slab gradient", dof=B - 1)


def _cornell_theta_scene(W):
    scene = workloads.cornell_scene(W, W)
    for m in range(3):
        scene["media"][m]["dyes"][0][1] *= 20
    return scene


def test_adjoint_vs_central_differences():
    """Camera scene (Cornell geometry and dyes): PRB gradient of a fixed
    positive functional vs central differences (h = 1e-3 relative) of the GPU
    forward render with common random numbers; 32 independent batches give
    the standard errors."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd.autograd import params_of, split_params
    W, n, B, h = 32, 1 << 20, 32, 1e-3
    scene = _cornell_theta_scene(W)
    theta = params_of(scene)
    sc = fpt.Scene(scene)
    rng = np.random.default_rng(9)
    g = torch.tensor(1.0 + rng.random(sc.film_shape()), dtype=torch.float32, device="cuda")
    prb = np.zeros((B, len(theta)))
    fd = np.zeros((B, len(theta)))
    for b in range(B):
        run = workloads.make_run(n, seed=1000 + b)
        prb[b] = sc.render_adjoint(run, g).cpu().numpy()
    for i in range(len(theta)):
        for sgn, store in ((+1, "p"), (-1, "m")):
            th = theta.copy()
            th[i] *= 1 + sgn * h
            sc.set_params(*split_params(scene, th))
            vals = []
            for b in range(B):
                f = sc.render(workloads.make_run(n, seed=1000 + b))
                vals.append(float((f.double() * g.double()).sum()))
            if store == "p":
                vp = np.array(vals)
            else:
                vm = np.array(vals)
        fd[:, i] = (vp - vm) / (2 * h * theta[i])
        sc.set_params(*split_params(scene, theta))
    sc.close()
    z, resolved = [], 0
    for i in range(len(theta)):
        se_p = prb[:, i].std(ddof=1) / math.sqrt(B)
        se = math.sqrt(se_p ** 2 + fd[:, i].var(ddof=1) / B)
        resolved += abs(prb[:, i].mean()) > 3 * se_p
        z.append((prb[:, i].mean() - fd[:, i].mean()) / se)
    print("prb", prb.mean(0) * theta, "fd", fd.mean(0) * theta, "z", np.round(z, 2))
    assert resolved >= 6
    check_z(z, "PRB vs central differences", dof=B - 1)


def test_autograd_l2_loss():
    """FluorRender in a torch graph: d/dtheta of sum((I - T)^2) through the
    autograd Function equals the adjoint seeded with 2 (I - T)."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd.autograd import params_of, render_differentiable
    W = 32
    scene = _cornell_theta_scene(W)
    target_scene = _cornell_theta_scene(W)
    for m, s in enumerate(workloads.ADJOINT_HIDDEN_CONC_SCALE):
        target_scene["media"][m]["dyes"][0][1] *= s
    n = 1 << 20
    target = fpt.Scene(target_scene).render(workloads.make_run(n, seed=1))
    sc = fpt.Scene(scene)
    theta = torch.tensor(params_of(scene), dtype=torch.float64, requires_grad=True)
    run = workloads.make_run(n, seed=0)
    film = render_differentiable(sc, theta, run)
    loss = ((film.double() - target.double()) ** 2).sum()
    loss.backward()
    g2 = sc.render_adjoint(run, (2 * (film.detach() - target)).float())
    torch.cuda.synchronize()
    np.testing.assert_allclose(theta.grad.numpy(), g2.cpu().numpy().astype(np.float64),
                               rtol=1e-5, atol=1e-9)
    # the concentration gradients point toward the hidden values
    gc = theta.grad.numpy()[:3]
    assert np.all(np.isfinite(theta.grad.numpy()))
    sc.close()
    print("dL/dc", gc)


def test_adjoint_full_size_memory_flat():
    """The adjoint of the full 256x256, 256 spp job runs with scratch memory
    that does not depend on the number of paths or their length."""
    import torch
    fpt = _fpt()
    scene, run, _, _ = workloads.adjoint_config()
    sc = fpt.Scene(scene)
    g = torch.ones(sc.film_shape(), device="cuda")
    free0 = torch.cuda.mem_get_info()[0]
    grad = sc.render_adjoint(run, g)
    torch.cuda.synchronize()
    free1 = torch.cuda.mem_get_info()[0]
    sc.close()
    assert np.all(np.isfinite(grad.cpu().numpy()))
    assert free0 - free1 < 64 << 20  # partial sums only, no per-path storage


def test_adjoint_full_size_sampled_replay():
    """The full 256x256, 256 spp adjoint job (2^24 paths): three sampled
    ranges of 4096 paths replay their records and per-path gradient
    contributions against the oracle over the first 256 vertices, and
    fpt_render_adjoint over one of those ranges equals the sum of its
    contributions and the oracle's gradient."""
    import torch
    fpt = _fpt()
    scene, run, _, _ = workloads.adjoint_config()
    g = _gfilm(scene)
    sc = fpt.Scene(scene)
    gt = torch.tensor(g, dtype=torch.float32, device="cuda")
    N = run["path_count"]
    for begin in (0, N // 2 + 17, N - 4096):
        sub = dict(run, path_begin=begin, path_count=4096)
        rec, rg = sc.records(sub, max_vertices=256, grad_film=gt)
        cond = oracle_replay(scene, sub, max_vertices=256, grad_film=g)
        print(compare_records(rec, cond, gpu_grad=rg))
    sub = dict(run, path_begin=N // 2 + 17, path_count=4096)
    rec, rg = sc.records(sub, grad_film=gt)
    total = sc.render_adjoint(sub, gt)
    torch.cuda.synchronize()
    sc.close()
    cond = oracle_replay(scene, sub, grad_film=g)
    print("full length", compare_records(rec, cond, gpu_grad=rg))
    print("total deviations", check_grad_total(total.cpu().numpy(), rg, cond))



def test_autograd_backward_uses_its_forward_parameters():
    """Two forwards through one scene at different theta, then backward of
    the first: the replay runs with the first theta (equal to
    fpt_render_adjoint at that theta up to the order of its fp32 partial sums,
    and far from the gradient at the second), and the scene keeps the
    second."""
    import torch
    fpt = _fpt()
    from paper_1706_03024_amd.autograd import params_of, render_differentiable, split_params
    scene = _cornell_theta_scene(16)
    run = workloads.make_run(1 << 18, seed=5)
    sc = fpt.Scene(scene)
    th1 = torch.tensor(params_of(scene), dtype=torch.float64, requires_grad=True)
    th2 = th1.detach().clone()
    th2[:3] *= 1.3   # the three concentrations
    th2.requires_grad_(True)
    f1 = render_differentiable(sc, th1, run)
    f2 = render_differentiable(sc, th2, run)
    g = torch.rand(f1.shape, generator=torch.Generator().manual_seed(9)).cuda()
    (f1 * g).sum().backward()
    got = th1.grad.numpy()
    assert np.array_equal(sc.theta, th2.detach().numpy())
    ref = fpt.Scene(scene)
    ref.set_params(*split_params(scene, th1.detach().numpy()))
    want = ref.render_adjoint(run, g.float().contiguous()).cpu().numpy().astype(np.float64)
    ref.set_params(*split_params(scene, th2.detach().numpy()))
    other = ref.render_adjoint(run, g.float().contiguous()).cpu().numpy().astype(np.float64)
    torch.cuda.synchronize()
    ref.close()
    np.testing.assert_allclose(got, want, rtol=1e-4, atol=1e-6 * np.abs(want).max())
    assert np.max(np.abs(other - want)) > 1e-2 * np.abs(want).max()
    assert not np.allclose(f1.detach().cpu().numpy(), f2.detach().cpu().numpy())
    sc.close()
