"""The seeded input generators (no GPU): the Fourier initial condition equals
its defining cosine sum, and the batch / serving workload draws are in range
and reproducible."""
import math

import numpy as np

from paper_1812_04789_amd import inputs


def test_fourier_field_equals_cosine_sum():
    ks, ph = inputs.fourier_phases(7)
    assert len(ks) == 9 ** 3 - 1
    x = np.random.default_rng(1).uniform(-1.0, 8.0, size=(40, 3))
    arg = x @ ks.T
    direct = np.stack([np.cos(arg + ph[:, c]).sum(-1) for c in range(3)], axis=-1)
    assert np.abs(inputs._fourier_raw(x, ks, ph, 2 * math.pi) - direct).max() < 1e-10
    # RMS scaling over the 16^3 sample grid
    g = (np.arange(16) + 0.5) * 2 * math.pi / 16
    G = np.stack(np.meshgrid(g, g, g, indexing='ij'), axis=-1).reshape(-1, 3)
    u = inputs.fourier_velocity(G, ks, ph, amp=0.1)
    assert abs(math.sqrt(np.mean(np.sum(u * u, axis=-1))) - 0.1) < 1e-12
    # periodic in the box
    assert np.allclose(inputs.fourier_velocity(x + 2 * math.pi, ks, ph), inputs.fourier_velocity(x, ks, ph),
                       atol=1e-11)


def test_batch_cases_draws():
    cs = inputs.batch_cases()
    assert len(cs) == 96 and cs == inputs.batch_cases()
    assert all(4 <= c["n"][0] <= 12 and c["n"][0] == c["n"][1] == c["n"][2] for c in cs)
    assert {c["p"] for c in cs} == {1, 2, 3, 4}
    assert all(0.05 <= c["mach"] <= 0.5 for c in cs)
    assert [c["seed"] for c in cs] == list(range(1812, 1812 + 96))


def test_serving_requests_draws():
    rq = inputs.serving_requests(count=500)
    t = np.array([r["t"] for r in rq])
    assert np.all(np.diff(t) > 0)
    assert abs(len(rq) / t[-1] - 200.0) < 30.0            # Poisson rate
    assert all(2 <= r["n"][0] <= 20 for r in rq)
    assert {r["p"] for r in rq} == {2, 3, 4}
    assert 0.35 < np.mean([r["mixed"] for r in rq]) < 0.65


def test_fourier_state_torch_equals_numpy():
    torch = __import__("torch")
    ks, ph = inputs.fourier_phases(9)
    x = np.random.default_rng(3).uniform(0.0, 2 * math.pi, size=(7, 11, 3))
    a = inputs.fourier_state(x, ks, ph, mach=0.2)
    b = inputs.fourier_state_torch(torch.tensor(x), ks, ph, mach=0.2, chunk=13).numpy()
    assert b.shape == a.shape
    assert np.abs(a - b).max() < 1e-9 * np.abs(a).max()
