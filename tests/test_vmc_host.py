"""Host-side pieces of the VMC loop (no GPU): the Adam step and the training appendix's schedules."""


def test_vmc_adam_matches_torch_adam():
    """The VMC loop's Adam step against torch.optim.Adam on the same gradients (CPU)."""
    import torch

    from paper_2605_13807_amd.vmc import Adam

    g = torch.Generator().manual_seed(0)
    th = torch.randn(50, generator=g)
    ref = th.clone().double().requires_grad_(True)
    opt_ref = torch.optim.Adam([ref], lr=1e-2)
    opt = Adam(50, "cpu", lr=1e-2)
    mine = th.clone().double()
    for _ in range(5):
        grad = torch.randn(50, generator=g, dtype=torch.float64)
        ref.grad = grad.clone()
        opt_ref.step()
        opt.step(mine, grad)
    assert torch.allclose(mine, ref.detach(), rtol=0, atol=1e-12)


def test_vmc_schedules():
    """Learning-rate decay and step-count rule of the training appendix, on values worked by hand."""
    from paper_2605_13807_amd.vmc import lr_decay, n_steps

    eta = lr_decay(5e-4, 5000)
    assert eta(0) == 5e-4 and abs(eta(5000) - 2.5e-4) < 1e-18 and abs(eta(15000) - 1.25e-4) < 1e-18
    # s = 1, C = 40000, r = 0.25, L0 = 6, F = 15000: 55000 steps at L = 6, 40000/e + 15000 = 29715.18 at L = 10
    assert n_steps(6, 1.0, 40000, 0.25, 6, 15000) == 55000
    assert n_steps(10, 1.0, 40000, 0.25, 6, 15000) == 29716
