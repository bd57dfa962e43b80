"""Differentiation through the projector (torch.autograd.Function whose
backward is the matched back projector), on the 64^3 crop of the uCT-shaped
workload: the adjoint test, linear finite differences, and central finite
differences through a nonlinear Beer-Lambert loss."""
import pytest
import torch

import synth

pytestmark = pytest.mark.gpu

DEV = torch.device("cuda", 0)


@pytest.fixture(scope="module")
def setup(gpu_lib):
    kct = gpu_lib
    from paper_2211_14212_amd import autograd as ag

    gd = synth.crop_geometry("muct1500", 64, 48, 32)
    plan = kct.Plan(kct.Geometry.from_dict(gd))
    x0 = torch.from_numpy(synth.phantom("muct1500", gd, full_n=1500, crop_origin=(718, 718, 718))).to(DEV)
    return kct, ag, plan, x0


def test_backward_is_matched_backprojector(setup):
    kct, ag, plan, x0 = setup
    x = x0.clone().requires_grad_(True)
    w = torch.randn(plan.geom.proj_shape, device=DEV, generator=torch.Generator(DEV).manual_seed(1))
    (ag.project(x, plan) * w).sum().backward()
    assert torch.equal(x.grad, plan.backproject(w))
    y = torch.randn(plan.geom.proj_shape, device=DEV, generator=torch.Generator(DEV).manual_seed(2))
    y.requires_grad_(True)
    v = torch.randn(plan.geom.vol_shape, device=DEV, generator=torch.Generator(DEV).manual_seed(3))
    (ag.backproject(y, plan) * v).sum().backward()
    assert torch.equal(y.grad, plan.forward(v))


def test_adjoint_identity_through_autograd(setup):
    kct, ag, plan, x0 = setup
    g = torch.Generator(DEV).manual_seed(4)
    x = torch.randn(plan.geom.vol_shape, device=DEV, generator=g).requires_grad_(True)
    w = torch.randn(plan.geom.proj_shape, device=DEV, generator=g)
    y = ag.project(x, plan)
    (y * w).sum().backward()
    lhs = float(torch.dot(y.detach().double().ravel(), w.double().ravel()))
    rhs = float(torch.dot(x.detach().double().ravel(), x.grad.double().ravel()))
    assert abs(lhs - rhs) <= 1e-6 * float(y.detach().double().norm() * w.double().norm())


def test_linear_finite_difference(setup):
    """A is linear: <w, A(x+hd) - A(x-hd)>/2h = <A^T w, d> up to rounding."""
    kct, ag, plan, x0 = setup
    g = torch.Generator(DEV).manual_seed(5)
    d = torch.randn(plan.geom.vol_shape, device=DEV, generator=g)
    w = torch.randn(plan.geom.proj_shape, device=DEV, generator=g)
    x = x0.clone().requires_grad_(True)
    (ag.project(x, plan) * w).sum().backward()
    h = 0.5
    fp = float((plan.forward(x0 + h * d).double() * w.double()).sum())
    fm = float((plan.forward(x0 - h * d).double() * w.double()).sum())
    fd = (fp - fm) / (2 * h)
    an = float((x.grad.double() * d.double()).sum())
    assert abs(fd - an) <= 1e-5 * (abs(an) + 1e-3 * abs(fp))


def test_nonlinear_loss_finite_difference(setup):
    """Beer-Lambert loss L(x) = || exp(-A x) - I/I0 ||^2, central differences
    along random directions against the autograd gradient."""
    kct, ag, plan, x0 = setup
    x = x0.clone().requires_grad_(True)
    target = torch.exp(-plan.forward(x0 * 0.9))

    def loss(v):
        return ((torch.exp(-ag.project(v, plan)) - target) ** 2).double().sum()

    loss(x).backward()
    g = torch.Generator(DEV).manual_seed(6)
    for _ in range(3):
        d = torch.randn(plan.geom.vol_shape, device=DEV, generator=g) * 0.05
        h = 1e-1
        with torch.no_grad():
            fd = (float(loss(x0 + h * d)) - float(loss(x0 - h * d))) / (2 * h)
        an = float((x.grad.double() * d.double()).sum())
        assert abs(fd - an) <= 2e-3 * abs(an) + 1e-6, (fd, an)
