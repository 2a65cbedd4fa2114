"""GPU parity of the hand-written adjoint (nb_force_vjp, nb_step_vjp, HermiteRun) against an
independent CPU FP64 autograd of the same discrete shared-step map and against FP64 finite
differences of the oracle."""
import numpy as np
import pytest
import torch

import oracle
from paper_astro_ph_0702058_amd import nbody
from paper_astro_ph_0702058_amd.adjoint import HermiteRun, SharedRunner
from paper_astro_ph_0702058_amd.plummer import perturb, plummer, sample_indices

pytestmark = pytest.mark.gpu


# ---- CPU FP64 autograd reference of the discrete map (Sec. 2 predictor, Eq. Force with App. A
# softening, corrector), written with plain torch operations
def torch_force(x, v, m, eps2):
    d = x[None, :, :] - x[:, None, :]            # d[i, j] = x_j - x_i
    u = v[None, :, :] - v[:, None, :]
    s = (d * d).sum(-1) + eps2
    off = ~torch.eye(x.shape[0], dtype=torch.bool)
    rinv = torch.where(off, s.clamp_min(1e-300).rsqrt(), torch.zeros_like(s))
    r3 = rinv ** 3
    r5 = rinv ** 5
    du = (d * u).sum(-1)
    a = (m[None, :, None] * d * r3[..., None]).sum(1)
    k = (m[None, :, None] * (u * r3[..., None] - 3 * du[..., None] * d * r5[..., None])).sum(1)
    return a, k


def torch_run(x0, v0, m, eps2, dt, nsteps):
    a, k = torch_force(x0, v0, m, eps2)
    x, v = x0, v0
    for _ in range(nsteps):
        xp = x + v * dt + a * dt ** 2 / 2 + k * dt ** 3 / 6
        vp = v + a * dt + k * dt ** 2 / 2
        a1, k1 = torch_force(xp, vp, m, eps2)
        a2 = -6 * (a - a1) / dt ** 2 - (4 * k + 2 * k1) / dt
        a3 = 12 * (a - a1) / dt ** 3 + 6 * (k + k1) / dt ** 2
        x = xp + a2 * dt ** 4 / 24 + a3 * dt ** 5 / 120
        v = vp + a2 * dt ** 3 / 6 + a3 * dt ** 4 / 24
        a, k = a1, k1
    return x, v


def soa(a):
    return torch.tensor(np.ascontiguousarray(np.asarray(a).T), dtype=torch.float64, device="cuda")


def gpu_grad(x0, v0, m, target, eps, dt, nsteps, ce, prec, overlap=True):
    runner = SharedRunner(len(m), eps, dt, nsteps, checkpoint_every=ce, precision=prec,
                          overlap=overlap)
    X0 = soa(x0).requires_grad_(True); V0 = soa(v0).requires_grad_(True)
    M = torch.tensor(m, dtype=torch.float64, device="cuda").requires_grad_(True)
    x, v = HermiteRun.apply(X0, V0, M, runner)
    loss = ((x - soa(target)) ** 2).sum(0).mean()
    loss.backward()
    return (float(loss.detach()), X0.grad.cpu().numpy().T, V0.grad.cpu().numpy().T, M.grad.cpu().numpy(),
            x.detach().cpu().numpy().T)


@pytest.mark.parametrize("prec,eps", [("fp64", 1 / 64), ("fp64", 0.0), ("fp32", 1 / 64),
                                      ("fp32", 0.0)])
def test_force_vjp_matches_autograd(prec, eps):
    """nb_force_vjp against autograd of the plain-torch force in FP64, at N = 300 (one whole
    and one ragged i-block; the self pair in a masked tile), softened (only the tile holding a
    particle's own slot tests for it) and unsoftened (every pair at zero separation skipped).
    FP64: 1e-11 of the largest component.  FP32 (float pair terms, tile sums in double): each
    pair term carries a few float roundings (about 1e-7 relative) and the largest terms come
    from the closest pairs, so 2e-6 of the largest component (printed: the measured error)."""
    n = 300
    x, v, m = plummer(n, 41)
    rng = np.random.default_rng(2)
    A = rng.normal(size=(n, 3)); B = rng.normal(size=(n, 3))
    xt = torch.tensor(x, requires_grad=True); vt = torch.tensor(v, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    a, k = torch_force(xt, vt, mt, eps * eps)
    ((a * torch.tensor(A)).sum() + (k * torch.tensor(B)).sum()).backward()
    st = nbody.DeviceState(x, v, m)
    with nbody.Context(n, eps, precision=prec) as ctx:
        ctx.nb_bind(st)
        ctx.nb_predict(torch.zeros(1, dtype=torch.int64, device="cuda"))
        xb = torch.zeros((3, n), dtype=torch.float64, device="cuda")
        vb = torch.zeros_like(xb); mb = torch.zeros(n, dtype=torch.float64, device="cuda")
        ctx.nb_force_vjp(soa(A), soa(B), xb, vb, mb)
        ctx.nb_sync()
    tol = 1e-11 if prec == "fp64" else 2e-6
    for name, got, ref in (("x", xb.cpu().numpy().T, xt.grad.numpy()),
                           ("v", vb.cpu().numpy().T, vt.grad.numpy()),
                           ("m", mb.cpu().numpy(), mt.grad.numpy())):
        err = np.max(np.abs(got - ref)) / np.max(np.abs(ref))
        print(f"{prec} eps={eps} {name}_bar: {err:.2e} of the largest component", flush=True)
        assert err <= tol, (name, err)


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_overlapped_backward_equals_sequential(prec):
    """The backward pass that recomputes the next segment on a second context and stream while
    the current segment's step VJPs run gives bitwise the gradients of the single-stream
    backward (the same kernels on the same inputs); 20 steps in segments of 8, 8 and 4."""
    n, eps, dt, nsteps, ce = 300, 1 / 64, 2.0 ** -8, 20, 8
    x0, v0, m = plummer(n, 44)
    xt, vt = perturb(x0, v0, 1e-3, 45)
    target = np.asarray(xt) + 0.01
    a = gpu_grad(x0, v0, m, target, eps, dt, nsteps, ce, prec, overlap=True)
    b = gpu_grad(x0, v0, m, target, eps, dt, nsteps, ce, prec, overlap=False)
    assert a[0] == b[0]
    for got, ref in zip(a[1:], b[1:]):
        assert np.array_equal(got, ref)


@pytest.mark.parametrize("ce", [1, 4, 5])
def test_run_gradient_fp64_matches_autograd(ce):
    """Whole run (12 shared steps, checkpoints every ce steps) in FP64 against CPU autograd of
    the same discrete map."""
    n, eps, dt, nsteps = 200, 1 / 32, 2.0 ** -8, 12
    x0, v0, m = plummer(n, 42)
    target = x0 + 0.01
    loss, gx, gv, gm, xf = gpu_grad(x0, v0, m, target, eps, dt, nsteps, ce, "fp64")
    xt = torch.tensor(x0, requires_grad=True); vt = torch.tensor(v0, requires_grad=True)
    mt = torch.tensor(m, requires_grad=True)
    x, _ = torch_run(xt, vt, mt, eps * eps, dt, nsteps)
    L = ((x - torch.tensor(target)) ** 2).sum(1).mean()
    L.backward()
    assert abs(loss - float(L)) <= 1e-12 * abs(float(L))
    for got, ref in ((gx, xt.grad.numpy()), (gv, vt.grad.numpy()), (gm, mt.grad.numpy())):
        assert np.max(np.abs(got - ref)) <= 1e-9 * np.max(np.abs(ref)), np.max(np.abs(got - ref))


# Error model of the gradient checks.  The FP64 gradient is compared with central finite
# differences of the FP64 oracle run; their floor is the finite differences' own error (rounding
# noise of a run, ~1e-9 absolute on the quotient, against the smallest sampled derivatives, and
# for the masses, varied by a relative step of 1e-3, the truncation error): TOL_FD = 1e-4 of the
# coordinate's scale.  The FP32 gradient (the same adjoint fed by single-precision forces and
# force VJPs) differs from the exact one by that same floor plus its arithmetic error, which is
# measured as its distance from the FP64 gradient of the same run and bounded by TOL_F32.  That
# error is a sum over steps and particles of the single-precision rounding of the forces and of
# the force VJPs, each within the FP32 force tolerance of its least accurate output, the jerk
# (1e-5 relative); the gradient inherits that relative bound.  Measured: 5.2e-7 (N = 1024) and
# 5.6e-7 (N = 16384) of the coordinate's scale.
TOL_FD = 1e-4
TOL_F32 = 1e-5


def _fd_errors(got, ref, fd_allow):
    """Per-coordinate error against the finite-difference reference, less the reference's own
    error estimate, over the coordinate's scale (floored at 1e-3 of the largest)."""
    scale = np.maximum(np.abs(ref), 1e-3 * np.max(np.abs(ref)))
    return np.maximum(np.abs(got - ref) - fd_allow, 0.0) / scale, scale


def _grad_at(gx, gv, gm, coords):
    return np.array([{"x": gx, "v": gv}[k][i, c] if k != "m" else gm[i] for k, i, c in coords])


def _check_gradient(prec, got, got64, ref, fd_allow, coords, label):
    err, scale = _fd_errors(got, ref, fd_allow)
    print(f"{label} {prec}: max rel err {err.max():.2e} over {len(coords)} coordinates "
          f"(largest raw {np.max(np.abs(got - ref) / scale):.2e})", flush=True)
    if prec == "fp64":
        assert err.max() <= TOL_FD, (err.max(), coords[int(np.argmax(err))])
        return
    d32 = np.abs(got - got64) / scale
    print(f"{label} fp32 against fp64 gradient of the same run: max {d32.max():.2e}", flush=True)
    assert d32.max() <= TOL_F32, (d32.max(), coords[int(np.argmax(d32))])
    assert err.max() <= TOL_FD + TOL_F32, (err.max(), coords[int(np.argmax(err))])


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_run_gradient_against_oracle_finite_differences(prec):
    """N = 1024 Plummer, eps = 1/128, 64 shared steps of 1/1024, checkpoints every 8; target =
    the end of an oracle run from initial conditions perturbed by N(0, 1e-3^2); loss = mean
    squared distance of the final positions.  The GPU gradient on 32 sampled coordinates of
    (x0, v0, m) against central FP64 finite differences of the oracle (error model above)."""
    n, eps, dt, nsteps = 1024, 1 / 128, 2.0 ** -10, 64
    x0, v0, m = plummer(n, 43)
    xp_, vp_ = perturb(x0, v0, 1e-3, 44)
    target, _ = oracle.shared_run(xp_, vp_, m, eps, dt, nsteps)
    loss, gx, gv, gm, xf = gpu_grad(x0, v0, m, target, eps, dt, nsteps, 8, prec)
    ref_loss = oracle.mean_sq_distance(oracle.shared_run(x0, v0, m, eps, dt, nsteps)[0], target)
    assert abs(loss - ref_loss) <= (1e-12 if prec == "fp64" else 1e-6) * ref_loss
    idx = sample_indices(n, 11, 45)
    coords = ([("x", int(i), int(i) % 3) for i in idx] + [("v", int(i), (int(i) + 1) % 3) for i in idx]
              + [("m", int(i), 0) for i in idx[:10]])
    fd = oracle.fd_gradient(x0, v0, m, eps, dt, nsteps, target, coords)
    got = _grad_at(gx, gv, gm, coords)
    got64 = None
    if prec == "fp32":
        got64 = _grad_at(*gpu_grad(x0, v0, m, target, eps, dt, nsteps, 8, "fp64")[1:4], coords)
    _check_gradient(prec, got, got64, fd, np.zeros_like(fd), coords, f"N={n}")


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_full_size_gradient_against_committed_finite_differences(prec):
    """The differentiable workload at full size: Plummer N = 16384, eps = 1/128, 64 shared steps
    of 1/1024, checkpoints every 8, loss = mean |x(T) - target|^2.  The GPU gradient at 32 sampled
    coordinates against the oracle's central finite differences committed in
    tests/golden/adjoint_fd.json (make_adjoint_reference.py).  The target is the GPU's FP64 run
    from the same perturbed initial conditions; it matches the oracle's (the stored coordinate
    sum to 1e-7, the loss to 1e-9 relative in FP64).  Error model as above; for the masses the
    reference is the Richardson value R = (4 D(h/2) - D(h)) / 3 from the relative steps h = 1e-2
    and h/2, and the allowance is |D(h) - D(h/2)| / 3, the estimate of the error of D(h/2) that
    R removes (R's own error is of higher order).  The larger mass step leaves a tenth of the
    rounding noise of the steps 1e-3 and 5e-4 (whose quotients differ by 2-4e-13 for every
    sampled mass, at derivatives down to 9e-10)."""
    import json
    import os
    path = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "adjoint_fd.json")
    if not os.path.exists(path):
        pytest.skip("the oracle finite differences have not been written")
    g = json.load(open(path))
    p = g["params"]
    n, eps, dt, nsteps = p["n"], p["eps"], p["dt"], p["nsteps"]
    x0, v0, m = plummer(n, p["seed"])
    xp_, vp_ = perturb(x0, v0, p["target_sigma"], p["target_seed"])
    runner = SharedRunner(n, eps, dt, nsteps, checkpoint_every=8, precision="fp64")
    with torch.no_grad():
        tx, _ = HermiteRun.apply(soa(xp_), soa(vp_), torch.tensor(m, device="cuda"), runner)
    target = tx.cpu().numpy().T.copy()
    assert abs(float(target.sum()) - g["target_sum"]) <= 1e-7
    loss, gx, gv, gm, xf = gpu_grad(x0, v0, m, target, eps, dt, nsteps, 8, prec)
    assert abs(loss - g["loss"]) <= (1e-9 if prec == "fp64" else 1e-5) * g["loss"]
    coords = [tuple(c) for c in g["coords"]]
    fd = np.array(g["fd"])
    ref = fd.copy()
    fd_allow = np.zeros_like(fd)
    wide = g["fd_mass_wide"]
    for c, d1, d2, r in zip(wide["coords"], wide["d_h"], wide["d_h2"], wide["richardson"]):
        k = coords.index(tuple(c))
        ref[k] = r
        fd_allow[k] = abs(d1 - d2) / 3.0
    assert all(c[0] != "m" or fd_allow[k] > 0 for k, c in enumerate(coords))
    got = _grad_at(gx, gv, gm, coords)
    got64 = None
    if prec == "fp32":
        got64 = _grad_at(*gpu_grad(x0, v0, m, target, eps, dt, nsteps, 8, "fp64")[1:4], coords)
    _check_gradient(prec, got, got64, ref, fd_allow, coords, f"N={n}")
