"""Checkpoints of the fitting loop, on the CPU: state_dict / load_state_dict
(and save / load through a file) carry the raw parameters, the children,
Adam's moments, the step count and the generator, so that a restored fit
takes exactly the steps the original takes.  Gradients are supplied by hand
here (the library's forward needs a GPU); tests/test_gpu_zfit.py resumes a
real run on the GPU."""

import numpy as np
import pytest

from paper_2405_20067_amd import inputs

torch = pytest.importorskip("torch")


def _fit(seed=0, **kw):
    from paper_2405_20067_amd.fit import Fit
    mix = inputs.gen_mixture(4, 12, seed=3)
    t = {a: torch.from_numpy(np.asarray(v, np.float32)) for a, v in mix.items()}
    return Fit(t["mean"], t["factor"], t["weight"], t["colour"], lr=1e-2, seed=seed, **kw)


def _fake_step(fit, rng):
    """One optimiser step with given gradients for every leaf."""
    fit.opt.zero_grad(set_to_none=True)
    for leaf in fit._leaves():
        leaf.grad = torch.from_numpy(rng.standard_normal(leaf.shape).astype(np.float32))
    fit.opt.step()
    fit.steps += 1


def _same(a, b):
    for x, y in zip(a._leaves(), b._leaves()):
        assert torch.equal(x.detach(), y.detach())
    assert a.steps == b.steps


def test_activated_start_is_the_given_mixture():
    from paper_2405_20067_amd.autograd import activate_factor
    mix = inputs.gen_mixture(4, 12, seed=3)
    fit = _fit()
    m, L, w, c = fit.absolute()
    np.testing.assert_allclose(L.detach().numpy(), mix["factor"], rtol=2e-6, atol=1e-7)
    np.testing.assert_allclose(w.detach().numpy(), mix["weight"], rtol=1e-6)
    assert torch.equal(activate_factor(fit.factor, 4), L)


@pytest.mark.parametrize("children", [False, True])
def test_resume_takes_the_same_steps(tmp_path, children):
    a = _fit(seed=7)
    if children:
        a.add_children()
    rng = np.random.default_rng(1)
    for _ in range(3):
        _fake_step(a, rng)
    path = str(tmp_path / "fit.pt")
    a.save(path)
    b = _fit(seed=99)          # another seed: the loaded generator must win
    b.load(path)
    _same(a, b)
    assert (b.child is None) == (not children)
    # the same later steps (including the generator's draws for new children)
    ra, rb = np.random.default_rng(5), np.random.default_rng(5)
    for _ in range(4):
        _fake_step(a, ra)
        _fake_step(b, rb)
    _same(a, b)
    ka, kb = a._default_children(3), b._default_children(3)
    for x, y in zip(ka, kb):
        assert torch.equal(x, y)


def test_checkpoint_holds_only_plain_tensors(tmp_path):
    a = _fit()
    a.add_children()
    _fake_step(a, np.random.default_rng(0))
    path = str(tmp_path / "fit.pt")
    a.save(path)
    st = torch.load(path, weights_only=True)
    assert all(torch.is_tensor(v) for v in st.values())
    assert st["steps"].item() == 1 and "adam.0.exp_avg" in st and "child.u" in st
