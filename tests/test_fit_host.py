"""Host-side logic of the Gauss-Newton refinement (``fit.lstsq_step``),
pinned to numpy's pseudo-inverse: the step is -pinv(J, rcond) r, exact for a
full-rank Jacobian and zero along the null directions of a rank-deficient
one (such as the common scale of D_DOM and the region factors)."""
import numpy as np
import torch

from paper_2406_04177_amd.fit import lstsq_step


def test_full_rank_step_solves_the_least_squares_problem():
    rng = np.random.default_rng(0)
    J = rng.standard_normal((40, 6))
    r = rng.standard_normal(40)
    d, sv = lstsq_step(torch.as_tensor(J), torch.as_tensor(r))
    ref = np.linalg.lstsq(J, -r, rcond=None)[0]
    np.testing.assert_allclose(d.numpy(), ref, rtol=1e-12, atol=1e-14)
    assert sv[0] == 1.0 and np.all(np.diff(sv.numpy()) <= 0)


def test_rank_deficient_step_leaves_the_null_direction():
    """Two columns enter only as their sum (as D_DOM and c_r enter as D c_r in
    log coordinates): the step is the minimum-norm solution, equal in the two
    coordinates, and it matches numpy's pseudo-inverse."""
    rng = np.random.default_rng(1)
    A = rng.standard_normal((30, 4))
    J = np.concatenate([A[:, :1], A], axis=1)     # columns 0 and 1 identical
    r = rng.standard_normal(30)
    d, sv = lstsq_step(torch.as_tensor(J), torch.as_tensor(r), rcond=1e-9)
    d = d.numpy()
    np.testing.assert_allclose(d, -np.linalg.pinv(J, rcond=1e-9) @ r, rtol=1e-10, atol=1e-13)
    assert abs(d[0] - d[1]) <= 1e-12 * abs(d).max()
    assert sv.numpy()[-1] < 1e-12
    # the residual after the step is the least-squares residual
    res = J @ d + r
    ref = A @ np.linalg.lstsq(A, -r, rcond=None)[0] + r
    np.testing.assert_allclose(res, ref, rtol=1e-10, atol=1e-12)


def test_gauss_newton_iteration_on_an_exponential_fit():
    """Plain Gauss-Newton iterations with lstsq_step on y = a exp(-b t) in log
    coordinates reach the generating (a, b) from 30 % away."""
    t = np.linspace(0.0, 3.0, 25)
    a, b = 2.0, 0.7
    y = a * np.exp(-b * t)
    la, lb = np.log(a * 1.3), np.log(b * 0.75)
    for _ in range(12):
        f = np.exp(la) * np.exp(-np.exp(lb) * t)
        J = np.stack([f, -np.exp(lb) * t * f], axis=1)
        d, _ = lstsq_step(torch.as_tensor(J), torch.as_tensor(f - y))
        la, lb = la + float(d[0]), lb + float(d[1])
    assert abs(np.exp(la) / a - 1) < 1e-12 and abs(np.exp(lb) / b - 1) < 1e-12


def test_default_tape_budget():
    """Every segment when all fit with a tenth of the free memory and two
    adjoint field sets to spare; else room is left for the checkpoints and
    the one segment recorded again in the backward; never negative."""
    from paper_2406_04177_amd.autograd import default_tape_bytes
    G = 1 << 30
    # 20 segments of 10 GiB, field set 1 GiB
    assert default_tape_bytes(300 * G, 10 * G, 200 * G, G, 20) == 200 * G
    # 250 GiB free: 25 + 2 spare, 10 for the re-recorded segment, 40 checkpoints
    assert default_tape_bytes(250 * G, 10 * G, 400 * G, G, 40) == 250 * G - 27 * G - 10 * G - 40 * G
    assert default_tape_bytes(20 * G, 10 * G, 400 * G, G, 40) == 0
