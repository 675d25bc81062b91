"""torch.autograd.Function over gm_integrate_grad: backward of a function of
the integral equals the chain rule applied to the adjoint gradient."""
from __future__ import annotations

import numpy as np
import pytest
import torch

import closed_forms as cf
from paper_2511_01573_amd import gm, workloads as W
from paper_2511_01573_amd.autograd import integral

pytestmark = pytest.mark.gpu


def test_autograd_chain_rule_gaussian():
    d = 3
    rng = np.random.default_rng(3)
    p = np.concatenate([rng.uniform(1, 4, d), rng.uniform(0.2, 0.8, d)])
    theta = torch.tensor(p, dtype=torch.float64, requires_grad=True)
    I = integral(theta, "gaussian", np.zeros(d), np.ones(d), 1e-9)
    loss = I * I
    loss.backward()
    _, _, g, _ = gm.integrate_grad("gaussian", p, np.zeros(d), np.ones(d), 1e-9)
    assert torch.allclose(theta.grad, torch.as_tensor(2 * I.item() * g), rtol=1e-14, atol=0)
    want = np.array([float(x) for x in cf.gaussian_grad(p[:d], p[d:])])
    assert np.abs(g - want).max() <= 1e-7 * np.abs(want).max()


def test_autograd_on_device_tensor():
    d = 4
    p = W.family_params(1, d, seed=9)
    theta = torch.tensor(p, dtype=torch.float64, device="cuda", requires_grad=True)
    I = integral(theta, "oscillatory", np.zeros(d), np.ones(d), 1e-8)
    I.backward()
    assert theta.grad.device.type == "cuda"
    assert torch.isfinite(theta.grad).all()
    exact_I = float(cf.exact(1, p[:d], p[d:]))
    assert abs(I.item() - exact_I) <= 1e-7 * max(abs(exact_I), 1e-3)
