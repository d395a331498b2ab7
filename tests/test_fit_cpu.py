"""Host logic of the staggered fitting driver (no GPU): the two losses'
derivatives against central differences, and its Adam against torch's."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
fit = pytest.importorskip("paper_2303_10440_amd.fit")


@pytest.mark.parametrize("loss_fn", ["weighted_l2", "plain_l2"])
def test_loss_derivative_matches_central_differences(loss_fn):
    fn = getattr(fit, loss_fn)
    rng = np.random.default_rng(3)
    t = torch.tensor(rng.random((3, 4, 5)) + 0.1, dtype=torch.float64)
    x = torch.tensor(rng.random((3, 4, 5)), dtype=torch.float64)
    loss, d = fn(x, t)
    h = 1e-6
    for idx in [(0, 0, 0), (1, 2, 3), (2, 3, 4)]:
        xp, xm = x.clone(), x.clone()
        xp[idx] += h
        xm[idx] -= h
        fd = (fn(xp, t)[0] - fn(xm, t)[0]) / (2 * h)
        assert abs(fd - float(d[idx])) < 1e-7 * max(1.0, abs(fd))
    if loss_fn == "weighted_l2":
        assert abs(loss - float(((x - t) ** 2 * t).sum() / t.sum())) < 1e-15
    else:
        assert abs(loss - float(((x - t) ** 2).mean())) < 1e-15


def test_adam_matches_torch_adam():
    rng = np.random.default_rng(5)
    x0 = torch.tensor(rng.standard_normal((7, 3)), dtype=torch.float64)
    grads = [torch.tensor(rng.standard_normal((7, 3)), dtype=torch.float64) for _ in range(6)]
    mine = x0.clone()
    opt = fit._Adam(mine, lr=0.05)
    ref = x0.clone().requires_grad_(True)
    topt = torch.optim.Adam([ref], lr=0.05, betas=(0.9, 0.999), eps=1e-8)
    for g in grads:
        opt.step(mine, g)
        ref.grad = g.clone()
        topt.step()
    assert torch.allclose(mine, ref.detach(), rtol=0, atol=1e-12)


def test_sigma6_and_psf_chain_rule():
    s = fit.sigma6(1.5, 3.0)
    assert s == (2.25, 2.25, 9.0, 0.0, 0.0, 0.0)


def test_adam_uniform_moves_every_entry_by_the_same_scale():
    rng = np.random.default_rng(6)
    x = torch.zeros((9, 3), dtype=torch.float64)
    g = torch.tensor(rng.standard_normal((9, 3)), dtype=torch.float64)
    opt = fit._AdamUniform(x, lr=0.1, eps=0.0)
    opt.step(x, g)
    # first step: m_hat = g, v_hat = g^2, so the step is lr g / max|g|
    assert torch.allclose(x, -0.1 * g / g.abs().max(), rtol=0, atol=1e-15)
