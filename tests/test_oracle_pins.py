"""Pins of the FP64 oracle against facts fixed by the paper and by
mathematics: closed forms, invariants, a library routine (SciPy's complex
spherical harmonics), central finite differences and brute force.  Each test
is chosen so that a plausible slip in the oracle (dropped term, wrong sign,
transposed index, wrong edge rule) fails it."""
import json
import math
import os

import numpy as np
import pytest
import scipy.special as sps

import synth
from oracle import oracle as O
from tests.oracle_util import dense_grid, lattice_coords, oracle_grid

HERE = os.path.dirname(os.path.abspath(__file__))


# ----------------------------------------------------------------------------
# Spherical harmonics (Sec. 3.2) against SciPy's complex harmonics


def _scipy_real_sh(d):
    """Real orthonormal SH of degree <= 2 from SciPy's complex Y_l^m (which
    carries the Condon-Shortley phase): sqrt2 Im Y_l^|m| for m<0, Y_l^0, and
    sqrt2 Re Y_l^m for m>0."""
    x, y, z = d
    theta = math.acos(max(-1.0, min(1.0, z)))
    phi = math.atan2(y, x)
    out = []
    for l in (0, 1, 2):
        for m in range(-l, l + 1):
            c = complex(sps.sph_harm_y(l, abs(m), theta, phi))
            if m < 0:
                out.append(math.sqrt(2.0) * c.imag)
            elif m == 0:
                out.append(c.real)
            else:
                out.append(math.sqrt(2.0) * c.real)
    return np.array(out)


def test_sh_basis_matches_scipy():
    rng = np.random.default_rng(0)
    d = rng.normal(size=(64, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ours = O.sh_basis(d)
    ref = np.stack([_scipy_real_sh(v) for v in d])
    np.testing.assert_allclose(ours, ref, rtol=0, atol=1e-13)


def test_sh_orthonormal_by_quadrature():
    # Gauss-Legendre in cos(theta) x uniform phi is exact for these degrees
    xg, wg = np.polynomial.legendre.leggauss(12)
    nphi = 16
    phis = (np.arange(nphi) + 0.5) * 2 * np.pi / nphi
    dirs, wts = [], []
    for ct, w in zip(xg, wg):
        st = math.sqrt(1 - ct * ct)
        for ph in phis:
            dirs.append((st * math.cos(ph), st * math.sin(ph), ct))
            wts.append(w * 2 * np.pi / nphi)
    Y = O.sh_basis(np.array(dirs))
    gram = (Y * np.array(wts)[:, None]).T @ Y
    np.testing.assert_allclose(gram, np.eye(9), atol=1e-12)


def test_sh_addition_theorem():
    rng = np.random.default_rng(1)
    d = rng.normal(size=(32, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    Y = O.sh_basis(d)
    np.testing.assert_allclose(Y[:, 0] ** 2, 1 / (4 * np.pi), rtol=1e-14)
    np.testing.assert_allclose((Y[:, 1:4] ** 2).sum(1), 3 / (4 * np.pi), rtol=1e-13)
    np.testing.assert_allclose((Y[:, 4:9] ** 2).sum(1), 5 / (4 * np.pi), rtol=1e-13)


# ----------------------------------------------------------------------------
# Ray extent and samples (Sec. 3.1; fixed step of half a voxel)


def test_axis_ray_extent_and_sample_count():
    n = 32
    g = dense_grid((n, n, n), np.ones(n ** 3), np.zeros((n ** 3, 27)))
    hit, tn, tf, ns = O.ray_extent(g, (-2.0, 0.0, 0.0), (1.0, 0.0, 0.0))
    assert hit
    # the lattice hull spans world x in [-0.5 + 0.5/n, 0.5 - 0.5/n]
    assert float(tn) == 2.0 - 0.5 + 0.5 / n
    assert float(tf) == 2.0 + 0.5 - 0.5 / n
    # half-voxel step: (n-1) voxels -> 2(n-1) samples
    assert ns == 2 * (n - 1)
    # a ray that passes beside the box misses it
    hit, _, _, ns = O.ray_extent(g, (-2.0, 0.9, 0.0), (1.0, 0.0, 0.0))
    assert not hit and ns == 0


def test_values_at_lattice_points_are_exact():
    n = 8
    rng = np.random.default_rng(2)
    dens = rng.uniform(0.5, 5.0, n ** 3)
    g = dense_grid((n, n, n), dens, np.zeros((n ** 3, 27)))
    # ray along +x through voxel centres j=3, k=5: every other sample sits on
    # a lattice point
    y = -0.5 + (3 + 0.5) / n
    z = -0.5 + (5 + 0.5) / n
    tr = O.trace_ray(g, (-2.0, y, z), (1.0, 0.0, 0.0))
    i, j, k = lattice_coords((n, n, n))
    lookup = {(a, b, c): v for a, b, c, v in zip(i, j, k, dens)}
    for s in range(0, len(tr["t"]), 2):
        cell = tuple(int(c) for c in tr["cell"][s])
        assert tr["sigma_pre"][s] == lookup[(cell[0], 3, 5)]


def test_trilinear_reproduces_affine_field():
    n = 10
    i, j, k = lattice_coords((n, n, n))
    a0, ax, ay, az = 2.0, 0.3, -0.2, 0.45
    dens = a0 + ax * i + ay * j + az * k + 5.0
    g = dense_grid((n, n, n), dens, np.zeros((n ** 3, 27)))
    o, d = synth.random_rays(16, seed=3, target_half=0.3)
    for r in range(16):
        tr = O.trace_ray(g, o[r].numpy(), d[r].numpy())
        t = tr["t"]
        p = o[r].double().numpy()[None, :] + t[:, None] * d[r].double().numpy()[None, :]
        gc = (p + 0.5) * n - 0.5  # grid coordinates in FP64
        expect = a0 + 5.0 + ax * gc[:, 0] + ay * gc[:, 1] + az * gc[:, 2]
        np.testing.assert_allclose(tr["sigma_pre"], expect, rtol=0, atol=2e-5)


# ----------------------------------------------------------------------------
# Compositing, Eq. (1)


def _y00():
    return complex(sps.sph_harm_y(0, 0, 0.3, 0.1)).real  # constant 1/(2 sqrt(pi))


def test_constant_density_closed_form_axis_ray():
    n, sigma = 16, 3.7
    kdc = np.array([0.9, 1.7, 2.4])
    sh = np.zeros((n ** 3, 27))
    sh[:, 0], sh[:, 9], sh[:, 18] = kdc
    g = dense_grid((n, n, n), np.full(n ** 3, sigma), sh)
    bg = np.array([1.0, 0.25, 0.5])
    rgb, tau, tf, ns = O.render_fwd(g, [[-2.0, 0.01, -0.02]], [[1.0, 0.0, 0.0]], bg)
    L = (n - 1) / n  # lattice hull length along x
    c = kdc * _y00()
    T = math.exp(-sigma * L)
    np.testing.assert_allclose(rgb[0], c * (1 - T) + bg * T, rtol=0, atol=1e-13)
    assert abs(tau[0] - sigma * L) < 1e-13
    assert abs(tf[0] - T) < 1e-14


def test_constant_density_closed_form_oblique_rays():
    n, sigma = 12, 2.3
    sh = np.zeros((n ** 3, 27))
    sh[:, 0] = sh[:, 9] = sh[:, 18] = 1.3
    g = dense_grid((n, n, n), np.full(n ** 3, sigma), sh)
    o, d = synth.random_rays(40, seed=5, target_half=0.2)
    rgb, tau, tf, _ = O.render_fwd(g, o.numpy(), d.numpy())
    lo, hi = -0.5 + 0.5 / n, 0.5 - 0.5 / n
    for r in range(40):
        oo, dd = o[r].double().numpy(), d[r].double().numpy()
        t0 = (lo - oo) / dd
        t1 = (hi - oo) / dd
        L = max(0.0, np.maximum(t0, t1).min() - max(0.0, np.minimum(t0, t1).max()))
        T = math.exp(-sigma * L)
        c = 1.3 * _y00()
        assert abs(tau[r] - sigma * L) < 1e-5 * sigma
        np.testing.assert_allclose(rgb[r], c * (1 - T) + T, atol=1e-5)


def test_zero_density_gives_background_and_no_sh_gradient():
    sv = synth.dense_random((6, 6, 6), seed=7)
    g = oracle_grid(sv)
    g.density[:] = 0.0
    o, d = synth.random_rays(32, seed=8)
    bg = (0.2, 0.4, 0.9)
    rgb, tau, tf, _ = O.render_fwd(g, o.numpy(), d.numpy(), bg)
    np.testing.assert_array_equal(rgb, np.tile(bg, (32, 1)))
    np.testing.assert_array_equal(tau, 0.0)
    gd, gs, touched = O.render_bwd(g, o.numpy(), d.numpy(), np.ones((32, 3)), bg)
    assert np.all(gs == 0.0) and np.all(gd == 0.0)
    assert touched.sum() > 0


def test_telescoping_weights_sum_to_one():
    # unit colour everywhere: C = sum_k w_k + T_n bg, so with bg = 0,
    # C + T_n = 1 (weights telescope); with bg = 1, C = 1.
    sh = np.zeros((512, 27))
    sh[:, 0] = sh[:, 9] = sh[:, 18] = 1.0 / _y00()
    g2 = dense_grid((8, 8, 8), np.random.default_rng(1).uniform(0.5, 30, 512), sh)
    o, d = synth.random_rays(50, seed=10)
    rgb, _, tf, ns = O.render_fwd(g2, o.numpy(), d.numpy(), (0.0, 0.0, 0.0))
    assert ns.max() > 0
    np.testing.assert_allclose(rgb + tf[:, None], 1.0, atol=1e-13)
    rgb1, _, _, _ = O.render_fwd(g2, o.numpy(), d.numpy(), (1.0, 1.0, 1.0))
    np.testing.assert_allclose(rgb1, 1.0, atol=1e-13)


def test_transmittance_monotone_and_miss_is_background():
    sv = synth.dense_random((8, 8, 8), seed=11)
    g = oracle_grid(sv)
    o = np.array([[-2.0, 0.9, 0.0], [-2.0, 0.0, 0.0]], np.float32)
    d = np.array([[1.0, 0.0, 0.0], [1.0, 0.0, 0.0]], np.float32)
    rgb, tau, tf, ns = O.render_fwd(g, o, d, (0.3, 0.6, 0.9))
    assert ns[0] == 0 and np.all(rgb[0] == np.array([0.3, 0.6, 0.9]))
    assert 0.0 < tf[1] < 1.0 and abs(tf[1] - math.exp(-tau[1])) < 1e-12


# ----------------------------------------------------------------------------
# Gradients: central finite differences of <G, C> and of the MSE loss


def _kink_margin(g, o, d):
    lo = np.inf
    for r in range(o.shape[0]):
        tr = O.trace_ray(g, o[r], d[r])
        sp = tr["sigma_pre"]
        rp = tr["rgb_pre"]
        live = sp > 0
        if live.any():
            lo = min(lo, sp[live].min(), np.abs(rp[live]).min())
    return lo


def _fd_check(g, o, d, G, bg, n_params, seed, tol=1e-6):
    gd, gs, touched = O.render_bwd(g, o, d, G, bg)

    def loss():
        return float((G * O.render_fwd(g, o, d, bg)[0]).sum())

    rng = np.random.default_rng(seed)
    ids = np.flatnonzero(touched)
    assert ids.size > 0
    checked = 0
    for m in rng.choice(ids, size=min(n_params, ids.size), replace=False):
        for q in (-1, int(rng.integers(0, 27))):
            arr, idx = (g.density, m) if q < 0 else (g.sh, (m, q))
            an = gd[m] if q < 0 else gs[m, q]
            x0 = arr[idx]
            h = 1e-6 * max(1.0, abs(x0))
            arr[idx] = x0 + h
            lp = loss()
            arr[idx] = x0 - h
            lm = loss()
            arr[idx] = x0
            fd = (lp - lm) / (2 * h)
            assert abs(fd - an) <= tol * abs(an) + 2e-8, (m, q, fd, an)
            checked += 1
    # untouched voxels get exactly zero gradient
    un = np.flatnonzero(touched == 0)
    assert np.all(gd[un] == 0) and np.all(gs[un] == 0)
    return checked


def test_fd_gradient_dense_grid():
    sv = synth.dense_random((6, 6, 6), seed=12, ho_scale=0.03)
    g = oracle_grid(sv)
    o, d = synth.random_rays(48, seed=13)
    o, d = o.numpy(), d.numpy()
    assert _kink_margin(g, o, d) > 1e-3
    G = np.random.default_rng(14).normal(size=(48, 3))
    assert _fd_check(g, o, d, G, (1.0, 1.0, 1.0), 40, 15) >= 60


def test_fd_gradient_sparse_grid_background():
    sv = synth.dense_random((8, 8, 8), seed=16, occupancy=0.55, sigma_lo=0.5,
                            sigma_hi=25.0, ho_scale=0.03)
    g = oracle_grid(sv)
    o, d = synth.random_rays(64, seed=17)
    o, d = o.numpy(), d.numpy()
    assert _kink_margin(g, o, d) > 1e-5
    G = np.random.default_rng(18).normal(size=(64, 3))
    _fd_check(g, o, d, G, (0.7, 0.2, 1.0), 40, 19, tol=1e-5)


def test_fd_gradient_random_direction_and_mse_chain():
    sv = synth.dense_random((5, 7, 6), seed=20, ho_scale=0.03)
    g = oracle_grid(sv)
    o, d = synth.random_rays(40, seed=21)
    o, d = o.numpy(), d.numpy()
    target = np.random.default_rng(22).uniform(0, 1, (40, 3))
    rgb = O.render_fwd(g, o, d)[0]
    grad_rgb, _ = O.mse_grad(rgb, target)
    gd, gs, _ = O.render_bwd(g, o, d, grad_rgb)
    rng = np.random.default_rng(23)
    vd = rng.normal(size=g.density.shape)
    vs = rng.normal(size=g.sh.shape)
    d0, s0 = g.density.copy(), g.sh.copy()
    h = 1e-6

    def mse():
        return O.mse_grad(O.render_fwd(g, o, d)[0], target)[1]

    g.density[:] = d0 + h * vd
    g.sh[:] = s0 + h * vs
    lp = mse()
    g.density[:] = d0 - h * vd
    g.sh[:] = s0 - h * vs
    lm = mse()
    g.density[:] = d0
    g.sh[:] = s0
    fd = (lp - lm) / (2 * h)
    an = float((gd * vd).sum() + (gs * vs).sum())
    assert abs(fd - an) <= 1e-6 * abs(an) + 1e-9


def test_relu_kinks_have_zero_derivative():
    # negative colour coefficients: clipped channels get no SH gradient
    sv = synth.dense_random((6, 6, 6), seed=24)
    g = oracle_grid(sv)
    g.sh[:, 0] = -5.0  # red always negative -> clipped to 0
    o, d = synth.random_rays(16, seed=25)
    rgb, *_ = O.render_fwd(g, o.numpy(), d.numpy(), (0.0, 0.0, 0.0))
    assert np.all(rgb[:, 0] == 0.0)
    _, gs, _ = O.render_bwd(g, o.numpy(), d.numpy(), np.ones((16, 3)), (0.0, 0.0, 0.0))
    assert np.all(gs[:, 0:9] == 0.0) and np.any(gs[:, 9:18] != 0.0)


def test_gradient_sums_do_not_depend_on_thread_count():
    # the gradient and its mass are summed in a fixed order (block order of
    # the rays), so one thread and all threads give the same bits, and a
    # second run repeats them
    sv = synth.dense_random((14, 12, 13), seed=26, occupancy=0.5)
    g = oracle_grid(sv)
    o, d = synth.random_rays(3000, seed=27)
    G = np.random.default_rng(28).normal(size=(3000, 3))
    n0 = O.max_threads()
    try:
        O.set_threads(1)
        a = O.render_bwd(g, o.numpy(), d.numpy(), G)
        ma = O.render_bwd_mass(g, o.numpy(), d.numpy(), np.abs(G))
        O.set_threads(max(n0, 3))
        b = O.render_bwd(g, o.numpy(), d.numpy(), G)
        c = O.render_bwd(g, o.numpy(), d.numpy(), G)
        mb = O.render_bwd_mass(g, o.numpy(), d.numpy(), np.abs(G))
    finally:
        O.set_threads(n0)
    for x, y, z in zip(a, b, c):
        assert np.array_equal(x, y) and np.array_equal(y, z)
    for x, y in zip(ma, mb):
        assert np.array_equal(x, y)


# ----------------------------------------------------------------------------
# Total variation (Sec. 3.5 and supplement B.1)


def test_tv_sh_linear_ramp_closed_form_and_telescoping():
    n, a, eps = 8, 0.7, 1e-9
    i, j, k = lattice_coords((n, n, n))
    sh = np.zeros((n ** 3, 27))
    sh[:, 5] = a * i  # ramp along x in one coefficient
    g = dense_grid((n, n, n), np.zeros(n ** 3), sh)
    loss, gd, gs, touched = O.tv(g, 0, n ** 3, 0.0, 1.0, eps)
    s = n / 256.0
    per_ramp = n * n * ((n - 1) * math.sqrt((s * a) ** 2 + eps) + math.sqrt(eps))
    per_flat = n ** 3 * math.sqrt(eps)
    assert abs(loss - (per_ramp + 26 * per_flat) / n ** 3) < 1e-12
    g5 = gs[:, 5].reshape(n, n, n)
    unit = s * (s * a) / math.sqrt((s * a) ** 2 + eps) / n ** 3
    np.testing.assert_allclose(g5[1:-1], 0.0, atol=1e-15)  # telescopes inside
    np.testing.assert_allclose(g5[0], -unit, rtol=1e-12)
    np.testing.assert_allclose(g5[-1], unit, rtol=1e-12)
    assert touched.all()


def test_tv_density_constant_field_edge_rule():
    # sigma: out-of-range neighbours read 0, so only cells on the upper faces
    # see a jump.  A cell on m upper faces has term sqrt(m (s c)^2 + eps).
    n, c, eps = 6, 2.5, 1e-9
    g = dense_grid((n, n, n), np.full(n ** 3, c), np.zeros((n ** 3, 27)))
    loss, gd, gs, _ = O.tv(g, 0, n ** 3, 1.0, 0.0, eps)
    s = n / 256.0
    expect = sum(math.comb(3, m) * (n - 1) ** (3 - m) * math.sqrt(m * (s * c) ** 2 + eps)
                 for m in range(4)) / n ** 3
    assert abs(loss - expect) < 1e-12
    assert np.all(gs == 0.0)


def test_tv_uniform_grid_is_finite_and_eps_must_be_positive():
    # the uniform initial grid: every SH difference is 0, so each SH term is
    # sqrt(eps) and its derivative 0 (finite only because eps > 0); eps = 0
    # is refused rather than dividing 0 by 0
    n, eps = 5, 1e-9
    sh = np.zeros((n ** 3, 27))
    sh[:, 0] = sh[:, 9] = sh[:, 18] = math.sqrt(math.pi)
    g = dense_grid((n, n, n), np.full(n ** 3, 0.1), sh)
    loss, gd, gs, touched = O.tv(g, 0, n ** 3, 0.0, 1.0, eps)
    assert np.all(np.isfinite(gs)) and np.all(gs == 0.0)
    assert abs(loss - 27 * math.sqrt(eps)) < 1e-15
    for bad in (0.0, -1e-9, float("nan")):
        with pytest.raises(ValueError):
            O.tv(g, 0, n ** 3, 1.0, 1.0, bad)


def test_tv_single_voxel_null_rules():
    n, c, eps = 7, 3.0, 1e-9
    mask = np.zeros(n ** 3, np.uint8)
    p = (3, 2, 4)
    mask[(p[0] * n + p[1]) * n + p[2]] = 1
    g = O.make_grid(np.array((n, n, n), np.int32), mask, np.array([c]),
                    np.random.default_rng(0).normal(size=(1, 27)))
    loss, gd, gs, touched = O.tv(g, 0, n ** 3, 1.0, 1.0, eps)
    s = n / 256.0
    # sigma: the voxel's own cell jumps on 3 axes, its 3 lower neighbours on
    # one axis, every other cell is flat; SH: one cell, all differences 0
    sig = (math.sqrt(3 * (s * c) ** 2 + eps) + 3 * math.sqrt((s * c) ** 2 + eps) +
           (n ** 3 - 4) * math.sqrt(eps))
    expect = (sig + 27 * math.sqrt(eps)) / n ** 3
    assert abs(loss - expect) < 1e-12
    # d/dc: own term -3 s (s(0-c))/term ... = +3 s^2 c/term_own, lower ones +s^2 c/term
    g_expect = (3 * s * s * c / math.sqrt(3 * (s * c) ** 2 + eps) +
                3 * s * s * c / math.sqrt((s * c) ** 2 + eps)) / n ** 3
    assert abs(gd[0] - g_expect) < 1e-12
    assert np.all(gs == 0.0) and touched[0] == 1


def test_tv_finite_differences_with_wraparound_segment():
    sv = synth.dense_random((6, 5, 7), seed=26, occupancy=0.6)
    g = oracle_grid(sv)
    ncell = 6 * 5 * 7
    start, count, eps = ncell - 50, 120, 1e-6  # wraps past the end
    _, gd, gs, touched = O.tv(g, start, count, 0.8, 1.3, eps)
    rng = np.random.default_rng(27)
    ids = np.flatnonzero(touched)
    for m in rng.choice(ids, size=25, replace=False):
        for q in (-1, int(rng.integers(0, 27))):
            arr, idx = (g.density, m) if q < 0 else (g.sh, (m, q))
            an = gd[m] if q < 0 else gs[m, q]
            x0 = arr[idx]
            h = 1e-6
            arr[idx] = x0 + h
            lp = O.tv(g, start, count, 0.8, 1.3, eps)[0]
            arr[idx] = x0 - h
            lm = O.tv(g, start, count, 0.8, 1.3, eps)[0]
            arr[idx] = x0
            fd = (lp - lm) / (2 * h)
            assert abs(fd - an) <= 1e-6 * abs(an) + 1e-10, (m, q, fd, an)


# ----------------------------------------------------------------------------
# RMSProp (Sec. 3.5)


def test_rmsprop_first_step_and_state_recurrence():
    m = 5
    rng = np.random.default_rng(28)
    dens = rng.normal(size=m)
    sh = rng.normal(size=(m, 27))
    gdn = rng.normal(size=m)
    gsh = rng.normal(size=(m, 27))
    vd = np.zeros(m)
    vs = np.zeros((m, 27))
    active = np.array([1, 0, 1, 1, 0], np.uint8)
    beta, eps, lr_s, lr_h = 0.95, 1e-8, 0.7, 0.01
    d0, s0, g0d, g0s = dens.copy(), sh.copy(), gdn.copy(), gsh.copy()
    O.rmsprop(active, dens, sh, vd, vs, gdn, gsh, lr_s, lr_h, beta, eps)
    on = active.astype(bool)
    np.testing.assert_allclose(
        dens[on], d0[on] - lr_s * g0d[on] / (math.sqrt(1 - beta) * np.abs(g0d[on]) + eps),
        rtol=1e-14)
    np.testing.assert_allclose(
        sh[on], s0[on] - lr_h * g0s[on] / (math.sqrt(1 - beta) * np.abs(g0s[on]) + eps),
        rtol=1e-14)
    # inactive voxels untouched bit for bit, active gradients cleared
    assert np.array_equal(dens[~on], d0[~on]) and np.array_equal(sh[~on], s0[~on])
    assert np.array_equal(gdn[~on], g0d[~on]) and np.all(gdn[on] == 0) and np.all(gsh[on] == 0)
    # constant gradient for t steps: v_t = (1 - beta^t) g^2
    for t in range(2, 7):
        gdn[:] = g0d
        gsh[:] = g0s
        O.rmsprop(np.ones(m, np.uint8), dens, sh, vd, vs, gdn, gsh, lr_s, lr_h, beta, eps)
    np.testing.assert_allclose(vd[~on], (1 - beta ** 5) * g0d[~on] ** 2, rtol=1e-13)
    np.testing.assert_allclose(vd[on], (1 - beta ** 6) * g0d[on] ** 2, rtol=1e-13)


def test_lr_schedules_match_paper_values():
    hp = json.load(open(os.path.join(HERE, "golden", "paper_hyperparams.json")))
    s, h = hp["lr_sigma"], hp["lr_sh"]
    assert abs(O.lr_schedule(0, h["lr0"], h["lr1"], h["max_steps"]) - 0.01) < 1e-15
    assert abs(O.lr_schedule(250000, h["lr0"], h["lr1"], h["max_steps"]) - 5e-6) < 1e-18
    end = O.lr_schedule(250000, s["lr0"], s["lr1"], s["max_steps"], s["delay_steps"], 0.01)
    assert abs(end - 0.05) < 1e-15
    # after the delay the sigma schedule is the plain exponential through 30
    mid = O.lr_schedule(125000, s["lr0"], s["lr1"], s["max_steps"], s["delay_steps"], 0.01)
    assert abs(mid - math.sqrt(30 * 0.05)) < 1e-12
    # at step 0 it starts at delay_mult * 30
    assert abs(O.lr_schedule(0, s["lr0"], s["lr1"], s["max_steps"], s["delay_steps"], 0.01)
               - 0.3) < 1e-14


# ----------------------------------------------------------------------------
# Grid create / prune / upsample (Sec. 3.4)


def test_create_is_storage_order_scan():
    rng = np.random.default_rng(29)
    mask = (rng.random(5 * 6 * 7) < 0.3).astype(np.uint8)
    index, m = O.grid_create((5, 6, 7), mask)
    assert m == mask.sum()
    occ = np.flatnonzero(mask)
    assert np.array_equal(index[occ], np.arange(m))
    assert np.all(index[mask == 0] == -1)


def _brute_keep(reso, index, density, thresh):
    nx, ny, nz = reso
    occ = np.zeros(reso, bool)
    idx = index.reshape(reso)
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                if idx[a, b, c] >= 0 and density[idx[a, b, c]] >= thresh:
                    occ[a, b, c] = True
    keep = np.zeros(reso, bool)
    for a in range(nx):
        for b in range(ny):
            for c in range(nz):
                if idx[a, b, c] < 0:
                    continue
                win = occ[max(a - 1, 0):a + 2, max(b - 1, 0):b + 2, max(c - 1, 0):c + 2]
                keep[a, b, c] = win.any()
    return keep.reshape(-1)


@pytest.mark.parametrize("seed", [30, 31, 32])
def test_prune_matches_brute_force(seed):
    reso = (6, 7, 5)
    sv = synth.dense_random(reso, seed=seed, occupancy=0.7, sigma_lo=0.0, sigma_hi=10.0)
    g = oracle_grid(sv)
    thresh = 8.5
    keep, kept, npr = O.prune_mask(g, thresh)
    bk = _brute_keep(reso, g.index, g.density, thresh)
    assert np.array_equal(keep.astype(bool), bk)
    assert kept == bk.sum() and kept + npr == g.n_vox
    g2, k2, p2 = O.prune(g, thresh)
    assert (k2, p2) == (kept, npr) and g2.n_vox == kept
    old = g.index[bk]
    np.testing.assert_array_equal(g2.density, g.density[old])


def test_prune_single_dense_voxel_survives_as_block():
    n = 7
    dens = np.full(n ** 3, 0.1)
    dens[(3 * n + 3) * n + 3] = 9.0
    dens[(0 * n + 0) * n + 6] = 9.0  # on a grid corner: 2x2x2 block
    g = dense_grid((n, n, n), dens, np.zeros((n ** 3, 27)))
    keep, kept, npr = O.prune_mask(g, 5.0)
    assert kept == 27 + 8 and npr == n ** 3 - 35


# ----------------------------------------------------------------------------
# MSI background (Sec. 3.6)

Y00 = 0.5 / math.sqrt(math.pi)


def _bg_grid(reso, density, coef):
    n = int(np.prod(reso))
    return O.bg_grid(reso, np.ones(n, np.uint8), density, coef)


def test_bg_tv_wraps_the_azimuth_closed_form():
    # colour coefficient k = column x in all three slots, constant along rows
    # and layers: only the azimuth differences count, (W/256) per step and
    # (W/256)(0 - (W-1)) from the last column back to the first
    L, H, W = 3, 4, 10
    l, y, x = np.meshgrid(np.arange(L), np.arange(H), np.arange(W), indexing="ij")
    g = _bg_grid((L, H, W), np.zeros(L * H * W), np.repeat(x.reshape(-1, 1).astype(float), 3, 1))
    n = L * H * W
    loss, gd, gs, touched = O.bg_tv(g, 0, n, 0.0, 1.0, 1e-14)
    expect = 3 * L * H * 2 * (W - 1) * (W / 256.0) / n
    assert abs(loss - expect) < 1e-9
    assert np.all(gs[:, :24] == 0) and np.all(gd == 0) and touched.all()
    # without the wrap the last column would add nothing: the plain TV of the
    # same values (colour slots 24-26 are SH slots there) is smaller
    loss_plain, _, gs_plain, _ = O.tv(g, 0, n, 0.0, 1.0, 1e-14)
    # (terms without a difference add sqrt(eps) = 1e-7 each: the 24 other SH
    # slots of every cell and the 3 colour slots of the last column)
    sq = (24 * n + 3 * L * H) * 1e-7
    assert abs(loss_plain - (3 * L * H * (W - 1) * (W / 256.0) + sq) / n) < 1e-9


def test_bg_tv_finite_differences():
    L, H, W = 4, 5, 6
    n = L * H * W
    rng = np.random.default_rng(18)
    mask = (rng.uniform(size=n) < 0.7).astype(np.uint8)
    m = int(mask.sum())
    g = O.bg_grid((L, H, W), mask, rng.uniform(0, 3, m), rng.uniform(-1, 2, (m, 3)))
    start, count, eps = n - 40, 90, 1e-6
    _, gd, gs, touched = O.bg_tv(g, start, count, 0.7, 1.1, eps)
    for mm in rng.choice(np.flatnonzero(touched), size=15, replace=False):
        for arr, idx, an in ((g.density, mm, gd[mm]), (g.sh, (mm, 24 + int(rng.integers(0, 3))), None)):
            an = gs[idx] if an is None else an
            x0 = arr[idx]
            h = 1e-6
            arr[idx] = x0 + h
            lp = O.bg_tv(g, start, count, 0.7, 1.1, eps)[0]
            arr[idx] = x0 - h
            lm = O.bg_tv(g, start, count, 0.7, 1.1, eps)[0]
            arr[idx] = x0
            assert abs((lp - lm) / (2 * h) - an) <= 1e-6 * abs(an) + 1e-10


def test_per_ray_background_colours():
    # C is affine in the background colour with slope T_final, per ray; a
    # per-ray colour array gives each ray what a call with its own colour does
    sv = synth.dense_random((7, 8, 6), seed=14, occupancy=0.5)
    g = oracle_grid(sv)
    o, d = synth.random_rays(12, seed=15)
    o, d = o.numpy(), d.numpy()
    bgs = np.random.default_rng(16).uniform(0, 1, (12, 3))
    rgb, _, tf, _ = O.render_fwd(g, o, d, bgs)
    rgb0, _, _, _ = O.render_fwd(g, o, d, (0.0, 0.0, 0.0))
    np.testing.assert_allclose(rgb, rgb0 + tf[:, None] * bgs, atol=1e-14)
    for r in (0, 5, 11):
        one, _, _, _ = O.render_fwd(g, o[r:r + 1], d[r:r + 1], bgs[r])
        np.testing.assert_array_equal(rgb[r], one[0])
    G = np.random.default_rng(17).normal(size=(12, 3))
    gd, gs, _ = O.render_bwd(g, o, d, G, bgs)
    for r in (2, 7):
        gd1, gs1, _ = O.render_bwd(g, o[r:r + 1], d[r:r + 1], G[r:r + 1], bgs[r])
        gd1b, gs1b, _ = O.render_bwd(g, o[r:r + 1], d[r:r + 1], G[r:r + 1], bgs[r:r + 1])
        np.testing.assert_array_equal(gd1, gd1b)
        np.testing.assert_array_equal(gs1, gs1b)


def test_bg_constant_closed_form_and_skipped_spheres():
    # constant opacity s and colour k: each of the 2(L-1) samples has
    # alpha = 1 - exp(-s/2), so C = Y00 k (1 - T) + T bg with T = exp(-s (L-1)),
    # from any origin inside the unit sphere in any direction
    L, H, W, s0 = 9, 8, 16, 0.7
    n = L * H * W
    k = np.array([1.0, 2.0, -3.0])
    g = _bg_grid((L, H, W), np.full(n, s0), np.tile(k, (n, 1)))
    o, d = synth.random_rays(20, seed=11, radius=0.6, target_half=0.2)
    bg = np.array([0.3, 0.5, 0.9])
    rgb, t = O.bg_render_fwd(g, o.numpy(), d.numpy(), bg)
    T = math.exp(-s0 * (L - 1))
    np.testing.assert_allclose(t, T, rtol=1e-12)
    np.testing.assert_allclose(rgb, np.tile(Y00 * np.maximum(k, 0) * (1 - T) + T * bg, (20, 1)), rtol=1e-12)
    # from outside the unit sphere the spheres that do not contain the origin
    # are skipped: sphere u has radius 1 / (1 - (u + 1/2)/L)
    r_o = 1.3
    u = 0.5 * np.arange(2 * (L - 1))
    inside = (1.0 / (1.0 - (u + 0.5) / L)) > r_o
    _, t2 = O.bg_render_fwd(g, [[0.0, 0.0, r_o]], [[0.0, 0.6, 0.8]], bg)
    assert abs(t2[0] - math.exp(-0.5 * s0 * inside.sum())) < 1e-12 and 0 < inside.sum() < u.size


def test_bg_equirectangular_lookup_and_wrap():
    # an opaque first sphere (u = 0 holds only layer 0) with colour
    # coefficient k(x, y) = x + 100 y: a ray from the centre sees the bilinear
    # texel mix at its own direction; phi = 0 sits between the last and the
    # first column (the image wraps), the poles clamp to the first/last row
    L, H, W = 4, 6, 12
    n = L * H * W
    l, y, x = np.meshgrid(np.arange(L), np.arange(H), np.arange(W), indexing="ij")
    dens = np.where(l.reshape(-1) == 0, 400.0, 0.0)
    kr = (x + 100.0 * y).reshape(-1).astype(np.float64)
    g = _bg_grid((L, H, W), dens, np.stack([kr, kr, kr], 1))
    dirs = np.array([[1.0, 0, 0], [0, 1.0, 0], [-1.0, 0, 0], [0, 0, 1.0], [0, 0, -1.0]])
    rgb, _ = O.bg_render_fwd(g, np.zeros((5, 3)), dirs, (0.0, 0.0, 0.0))
    mid = 100.0 * (H / 2 - 0.5)  # the equator lies between rows H/2-1 and H/2
    expect = [((W - 1) + 0) / 2 + mid, (W / 4 - 1 + W / 4) / 2 + mid, (W / 2 - 1 + W / 2) / 2 + mid, None, None]
    a = 1.0 - math.exp(-200.0)
    for i in range(3):
        assert abs(rgb[i, 0] - a * Y00 * expect[i]) < 1e-9, i
    # at the poles every column of the clamped row mixes in; the azimuth of a
    # pole direction is atan2(0, 0) = 0 (phi = 0: the wrap columns)
    assert abs(rgb[3, 0] - a * Y00 * ((W - 1) / 2 + 0.0)) < 1e-9
    assert abs(rgb[4, 0] - a * Y00 * ((W - 1) / 2 + 100.0 * (H - 1))) < 1e-9


def test_bg_fd_gradient():
    L, H, W = 5, 6, 10
    n = L * H * W
    rng = np.random.default_rng(12)
    dens = rng.uniform(0.0, 3.0, n)
    coef = rng.uniform(-1.0, 3.0, (n, 3))
    g = _bg_grid((L, H, W), dens, coef)
    o, d = synth.random_rays(25, seed=13, radius=0.5, target_half=0.3)
    o, d = o.numpy(), d.numpy()
    bg = np.array([0.2, 0.7, 0.4])
    G = rng.normal(size=(25, 3))
    gd, gs, touched = O.bg_render_bwd(g, o, d, G, bg)
    assert np.all(gs[:, :24] == 0)

    def loss():
        return float((G * O.bg_render_fwd(g, o, d, bg)[0]).sum())

    ids = np.flatnonzero(touched)
    assert ids.size > 50
    for m in rng.choice(ids, size=10, replace=False):
        for arr, idx, an in ((g.density, m, gd[m]), (g.sh, (m, 24 + int(rng.integers(0, 3))), None)):
            if an is None:
                an = gs[idx]
            x0 = arr[idx]
            h = 1e-6 * max(1.0, abs(x0))
            arr[idx] = x0 + h
            lp = loss()
            arr[idx] = x0 - h
            lm = loss()
            arr[idx] = x0
            assert abs((lp - lm) / (2 * h) - an) <= 1e-6 * abs(an) + 1e-8, (m, idx)
    assert np.all(gd[touched == 0] == 0) and np.all(gs[touched == 0] == 0)
    # the absolute-term mass dominates the gradient and equals it where no
    # terms cancel (colour slots with a positive upstream gradient)
    md, ms = O.bg_render_bwd_mass(g, o, d, np.abs(G), bg)
    assert np.all(md >= np.abs(gd) * (1 - 1e-12)) and np.all(ms >= np.abs(gs) * (1 - 1e-12))
    gp, sp, _ = O.bg_render_bwd(g, o, d, np.abs(G), bg)
    np.testing.assert_allclose(sp, ms, rtol=1e-12, atol=1e-300)


# ----------------------------------------------------------------------------
# NDC warp of forward-facing scenes (Sec. 3.6)


def _ndc_point(p, W, H, f, near):
    return np.array([-(2 * f / W) * p[0] / p[2], -(2 * f / H) * p[1] / p[2], 1 + 2 * near / p[2]])


def test_ndc_reference_camera_rays_are_parallel_to_z():
    # pixel (px, py) of the reference camera starts at NDC
    # ((px + 0.5 - W/2)/(W/2), -(py + 0.5 - H/2)/(H/2), -1) and runs along +z
    W, H, f, near = 40, 30, 33.0, 1.0
    c2w = np.array([[1.0, 0, 0, 0], [0, 1.0, 0, 0], [0, 0, 1.0, 0]])
    o, d = O.camera_rays(c2w, f, W, H)
    on, dn = O.rays_to_ndc(o, d, W, H, f, near)
    px, py = np.meshgrid(np.arange(W), np.arange(H))
    ex = (px.reshape(-1) + 0.5 - W / 2) / (W / 2)
    ey = -(py.reshape(-1) + 0.5 - H / 2) / (H / 2)
    np.testing.assert_allclose(on[:, 0], ex, atol=2e-6)
    np.testing.assert_allclose(on[:, 1], ey, atol=2e-6)
    np.testing.assert_allclose(on[:, 2], -1.0, atol=1e-6)
    np.testing.assert_allclose(np.abs(dn), np.tile([0.0, 0.0, 1.0], (W * H, 1)), atol=2e-6)
    assert np.all(dn[:, 2] > 0)


def test_ndc_maps_world_points_onto_the_ray_in_order():
    # the NDC images of the points of a world ray lie on the NDC ray, in the
    # same order, and tend to z = 1 far away
    W, H, f, near = 64, 48, 52.0, 1.0
    rng = np.random.default_rng(5)
    n = 60
    o = np.column_stack([rng.uniform(-0.3, 0.3, n), rng.uniform(-0.2, 0.2, n), rng.uniform(-0.2, 0.4, n)])
    d = np.column_stack([rng.uniform(-0.4, 0.4, n), rng.uniform(-0.3, 0.3, n), rng.uniform(-1.0, -0.5, n)])
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    o32, d32 = o.astype(np.float32), d.astype(np.float32)
    on, dn = O.rays_to_ndc(o32, d32, W, H, f, near)
    for r in range(n):
        oo, dd = o32[r].astype(np.float64), d32[r].astype(np.float64)
        t0 = -(near + oo[2]) / dd[2]
        prev = -np.inf
        for t in t0 + np.array([0.0, 0.3, 1.0, 4.0, 30.0, 1e4]):
            P = _ndc_point(oo + t * dd, W, H, f, near)
            rel = P - on[r].astype(np.float64)
            s = rel @ dn[r]
            assert np.linalg.norm(rel - s * dn[r]) < 1e-5 * (1 + abs(s)), (r, t)
            assert s > prev - 1e-6
            prev = s
        assert abs(P[2] - 1.0) < 1e-3
    # a ray parallel to the near plane never reaches it
    zo, zd = O.rays_to_ndc([[0.1, 0.2, 0.0]], [[1.0, 0.0, 0.0]], W, H, f, near)
    assert np.all(zo == 0) and np.all(zd == 0)


def test_ndc_centre_ray_and_near_plane():
    on, dn = O.rays_to_ndc([[0.0, 0.0, 0.0], [0.0, 0.0, 3.0]], [[0.0, 0.0, -1.0]] * 2, 80, 60, 70.0, 2.0)
    np.testing.assert_array_equal(on, [[0.0, 0.0, -1.0]] * 2)
    np.testing.assert_array_equal(np.abs(dn), [[0.0, 0.0, 1.0]] * 2)


# ----------------------------------------------------------------------------
# Sparsity (Cauchy) and beta priors (Sec. 3.7)


def test_regularisers_constant_density_axis_ray_closed_form():
    # 2(n-1) samples, all with density s, h = 1/(2n), L = (n-1)/n, T = exp(-s L).
    # Every sample's density gradient is t_s + t_b with t_s = lam_s 4s/(1+2s^2)
    # and t_b = -h T lam_b (1/(eps+T) - 1/(eps+1-T)); along x a voxel collects
    # trilinear weight 2 (1.5 at x = 0, 0.5 at x = n-1), across the ray the
    # bilinear weights of the offsets (0.25, 0.5).
    n, sig, lam_s, lam_b, eps = 16, 1.7, 0.3, 0.2, 1e-3
    g = dense_grid((n, n, n), np.full(n ** 3, sig), np.zeros((n ** 3, 27)))
    o, d = _axis_ray(n, 5.25, 9.5)
    ls, lb, gd, md = O.regularisers(g, o, d, lam_s, lam_b, eps)
    h, L = 0.5 / n, (n - 1) / n
    T = math.exp(-sig * L)
    assert abs(ls - lam_s * 2 * (n - 1) * math.log1p(2 * sig * sig)) < 1e-12
    assert abs(lb - lam_b * (math.log(eps + T) + math.log(eps + 1 - T))) < 1e-12
    t = lam_s * 4 * sig / (1 + 2 * sig * sig) - h * T * lam_b * (1 / (eps + T) - 1 / (eps + 1 - T))
    wx = np.full(n, 2.0)
    wx[0], wx[-1] = 1.5, 0.5
    expect = np.zeros((n, n, n))
    for jj, wy in ((5, 0.75), (6, 0.25)):
        for kk, wz in ((9, 0.5), (10, 0.5)):
            expect[:, jj, kk] = wx * wy * wz * t
    got = np.zeros(n ** 3)
    got[g.index >= 0] = gd[g.index[g.index >= 0]]
    np.testing.assert_allclose(got.reshape(n, n, n), expect, rtol=1e-12, atol=1e-15)
    assert np.all(md >= np.abs(gd) - 1e-15)


def test_regularisers_fd_gradient_sparse_grid():
    sv = synth.dense_random((7, 6, 8), seed=71, occupancy=0.6, sigma_lo=0.2, sigma_hi=30.0)
    g = oracle_grid(sv)
    o, d = synth.random_rays(40, seed=72)
    o, d = o.numpy(), d.numpy()
    lam_s, lam_b, eps = 0.05, 0.3, 1e-3
    _, _, gd, md = O.regularisers(g, o, d, lam_s, lam_b, eps)

    def loss():
        a, b, _, _ = O.regularisers(g, o, d, lam_s, lam_b, eps)
        return a + b

    rng = np.random.default_rng(73)
    ids = np.flatnonzero(gd != 0)
    assert ids.size > 10
    for m in rng.choice(ids, size=12, replace=False):
        x0 = g.density[m]
        hh = 1e-6 * max(1.0, abs(x0))
        g.density[m] = x0 + hh
        lp = loss()
        g.density[m] = x0 - hh
        lm = loss()
        g.density[m] = x0
        fd = (lp - lm) / (2 * hh)
        assert abs(fd - gd[m]) <= 1e-5 * abs(gd[m]) + 1e-9, (m, fd, gd[m])
    assert np.all(md >= np.abs(gd) * (1 - 1e-12))


def test_regularisers_relu_and_beta_signs():
    n = 8
    o, d = _axis_ray(n, 3.5, 4.25)
    # negative densities: clipped, no Cauchy loss and no gradient; T = 1 gives
    # the constant beta loss of an empty ray
    g = dense_grid((n, n, n), np.full(n ** 3, -2.0), np.zeros((n ** 3, 27)))
    ls, lb, gd, _ = O.regularisers(g, o, d, 1.0, 1.0, 1e-3)
    assert ls == 0.0 and np.all(gd == 0.0)
    assert abs(lb - (math.log(1.001) + math.log(1e-3))) < 1e-12
    # a miss contributes the same constant and nothing else
    ls2, lb2, gd2, _ = O.regularisers(g, [[5.0, 5.0, 5.0]], [[1.0, 0.0, 0.0]], 1.0, 1.0, 1e-3)
    assert ls2 == 0.0 and lb2 == lb and np.all(gd2 == 0.0)
    # beta alone: a mostly transparent ray (T > 1/2) is pushed to empty (positive
    # density gradient), a mostly opaque one (T < 1/2) to opaque (negative)
    for sig, sign in ((0.3, 1.0), (40.0, -1.0)):
        g = dense_grid((n, n, n), np.full(n ** 3, sig), np.zeros((n ** 3, 27)))
        _, _, gd, _ = O.regularisers(g, o, d, 0.0, 1.0, 1e-3)
        nz = gd[gd != 0]
        assert nz.size > 0 and np.all(np.sign(nz) == sign)


# ----------------------------------------------------------------------------
# Pruning by weight (Sec. 3.4): per-voxel maximum of the compositing weight


def _axis_ray(n, gy, gz):
    """+x ray whose grid coordinates across the axis are (gy, gz)."""
    return [[-2.0, (gy + 0.5) / n - 0.5, (gz + 0.5) / n - 0.5]], [[1.0, 0.0, 0.0]]


def test_max_weight_constant_density_axis_ray_closed_form():
    # Constant density: sample k sits at grid x = k/2 in cell floor(k/2) and
    # every interval is h = 1/(2n) world units, so w_k = exp(-s k h)(1 - exp(-s h)),
    # decreasing in k.  Voxel x is a corner of cells x-1 and x, whose first
    # sample is k = 2 max(x-1, 0); only the 4 voxel lines around the ray see it.
    n, sig = 16, 3.7
    g = dense_grid((n, n, n), np.full(n ** 3, sig), np.zeros((n ** 3, 27)))
    o, d = _axis_ray(n, 5.3, 9.6)
    w = O.max_weight(g, o, d)
    h = 0.5 / n
    expect = np.zeros((n, n, n))
    for x in range(n):
        k = 2 * max(x - 1, 0)
        expect[x, 5:7, 9:11] = math.exp(-sig * k * h) * (1.0 - math.exp(-sig * h))
    got = np.zeros(n ** 3)
    got[g.index >= 0] = w[g.index[g.index >= 0]]
    np.testing.assert_allclose(got.reshape(n, n, n), expect, rtol=1e-12, atol=0)


def test_max_weight_peaks_at_a_surface():
    # Density 0 for voxels x < s and S from x = s on: along the axis ray the
    # interpolated density is 0 up to grid x = s-1, rises linearly to S over
    # cell s-1 and stays S.  The weights rise, peak just inside the surface and
    # fall, so the maximum is not the first sample's weight (a "first" or "sum"
    # reduction fails here), and voxels before the surface see only zero.  (n a
    # power of two keeps the FP32 sample positions at exactly k/2.)
    n, s, S = 16, 6, 40.0
    i, j, k = lattice_coords((n, n, n))
    g = dense_grid((n, n, n), np.where(i >= s, S, 0.0), np.zeros((n ** 3, 27)))
    o, d = _axis_ray(n, 3.25, 7.5)
    w = O.max_weight(g, o, d)
    h = 0.5 / n
    xs = 0.5 * np.arange(2 * (n - 1))
    sig = np.clip(xs - (s - 1), 0.0, 1.0) * S
    tau_before = np.concatenate([[0.0], np.cumsum(sig * h)[:-1]])
    wk = np.exp(-tau_before) * (1.0 - np.exp(-sig * h))
    cell = np.floor(xs).astype(int)
    expect = np.zeros((n, n, n))
    for x in range(n):
        near = (cell == x) | (cell == x - 1)
        expect[x, 3:5, 7:9] = wk[near].max() if near.any() else 0.0
    got = np.zeros(n ** 3)
    got[g.index >= 0] = w[g.index[g.index >= 0]]
    np.testing.assert_allclose(got.reshape(n, n, n), expect, rtol=1e-12, atol=1e-300)
    peak = int(np.argmax(expect[:, 3, 7]))
    assert expect[peak, 3, 7] > expect[peak + 2, 3, 7] > 0 and expect[s - 2, 3, 7] == 0.0


def test_max_weight_is_a_maximum_over_rays_and_bounded_by_opacity():
    sv = synth.dense_random((9, 8, 10), seed=41, occupancy=0.5, sigma_lo=0.0, sigma_hi=40.0)
    g = oracle_grid(sv)
    o, d = synth.random_rays(120, seed=42)
    o, d = o.numpy(), d.numpy()
    w_all = O.max_weight(g, o, d)
    w_a = O.max_weight(g, o[:50], d[:50])
    w_b = O.max_weight(g, o[50:], d[50:])
    # accumulation over batches is the element-wise maximum, not a sum
    np.testing.assert_array_equal(w_all, np.maximum(w_a, w_b))
    acc = O.max_weight(g, o[:50], d[:50])
    O.max_weight(g, o[50:], d[50:], acc)
    np.testing.assert_array_equal(acc, w_all)
    # w_k <= sum_k w_k = 1 - T_final of its ray; a voxel is seen only by
    # samples that read it, so the set with a non-zero maximum lies inside the
    # touched set of the gradient pass
    _, _, tf, _ = O.render_fwd(g, o, d)
    assert w_all.max() <= (1.0 - tf).max() + 1e-15
    _, _, touched = O.render_bwd(g, o, d, np.ones((120, 3)))
    assert np.all(touched[w_all > 0] == 1) and (w_all > 0).sum() > 20
    # one ray at a time: the largest voxel value is that ray's largest weight
    for r in range(10):
        wr = O.max_weight(g, o[r:r + 1], d[r:r + 1])
        tr = O.trace_ray(g, o[r], d[r])
        sig = np.maximum(tr["sigma_pre"], 0.0)
        tau = np.concatenate([[0.0], np.cumsum(sig * tr["delta"])[:-1]])
        wk = np.exp(-tau) * -np.expm1(-sig * tr["delta"])
        assert abs(wr.max() - (wk.max() if len(wk) else 0.0)) < 1e-12


@pytest.mark.parametrize("seed", [33, 34])
def test_prune_by_weight_matches_brute_force(seed):
    reso = (7, 6, 6)
    sv = synth.dense_random(reso, seed=seed, occupancy=0.6)
    g = oracle_grid(sv)
    vals = np.random.default_rng(seed).uniform(0.0, 1.0, g.n_vox)
    thresh = 0.9
    keep, kept, npr = O.prune_mask(g, thresh, vals)
    bk = _brute_keep(reso, g.index, vals, thresh)
    assert np.array_equal(keep.astype(bool), bk)
    assert kept == bk.sum() and kept + npr == g.n_vox
    g2, k2, p2 = O.prune(g, thresh, vals)
    assert (k2, p2) == (kept, npr)
    np.testing.assert_array_equal(g2.density, g.density[g.index[bk]])


def test_upsample_affine_exact_and_counts():
    n, n2 = 6, 12
    i, j, k = lattice_coords((n, n, n))
    dens = 1.0 + 0.5 * i - 0.25 * j + 0.125 * k + 3.0
    sh = np.stack([0.1 * q + 0.3 * i - 0.2 * k for q in range(27)], axis=1)
    g = dense_grid((n, n, n), dens, sh)
    g2 = O.upsample(g, (n2, n2, n2))
    assert g2.n_vox == n2 ** 3
    I, J, K = lattice_coords((n2, n2, n2))
    gx = (I + 0.5) * n / n2 - 0.5
    gy = (J + 0.5) * n / n2 - 0.5
    gz = (K + 0.5) * n / n2 - 0.5
    inside = (gx >= 0) & (gx <= n - 1) & (gy >= 0) & (gy <= n - 1) & (gz >= 0) & (gz <= n - 1)
    exp_d = 4.0 + 0.5 * gx - 0.25 * gy + 0.125 * gz
    np.testing.assert_allclose(g2.density[inside], exp_d[inside], atol=1e-13)
    np.testing.assert_allclose(g2.sh[inside, 4], (0.4 + 0.3 * gx - 0.2 * gz)[inside], atol=1e-13)


def test_upsample_identity_ratio_and_children_of_one_voxel():
    sv = synth.dense_random((5, 6, 4), seed=33, occupancy=0.5)
    g = oracle_grid(sv)
    g1 = O.upsample(g, (5, 6, 4))
    assert np.array_equal(g1.index, g.index)
    # same resolution: values at lattice points are reproduced (NULL = 0 only
    # enters through zero weights)
    np.testing.assert_array_equal(g1.density, g.density)
    # one occupied voxel, ratio 4 -> a 4x4x4 block of children
    n = 4
    mask = np.zeros(n ** 3, np.uint8)
    mask[(1 * n + 2) * n + 3] = 1
    go = O.make_grid(np.array((n,) * 3, np.int32), mask, np.array([2.0]), np.zeros((1, 27)))
    gu = O.upsample(go, (16, 16, 16))
    assert gu.n_vox == 64
    occ = np.flatnonzero(gu.index >= 0)
    I, J, K = occ // 256, (occ // 16) % 16, occ % 16
    assert set(I) == {4, 5, 6, 7} and set(J) == {8, 9, 10, 11} and set(K) == {12, 13, 14, 15}


def test_upsample_non_integer_ratio_counts_brute_force():
    sv = synth.dense_random((6, 5, 7), seed=34, occupancy=0.4)
    g = oracle_grid(sv)
    new = (9, 8, 10)
    gu = O.upsample(g, new)
    idx = g.index.reshape(6, 5, 7)
    cnt = 0
    for a in range(new[0]):
        for b in range(new[1]):
            for c in range(new[2]):
                pa = int(math.floor((a + 0.5) * 6 / new[0]))
                pb = int(math.floor((b + 0.5) * 5 / new[1]))
                pc = int(math.floor((c + 0.5) * 7 / new[2]))
                cnt += idx[pa, pb, pc] >= 0
    assert gu.n_vox == cnt


def test_gradient_mass_bounds_gradient_and_is_tight_without_cancellation():
    sv = synth.dense_random((7, 6, 8), seed=35, occupancy=0.6, ho_scale=0.2)
    g = oracle_grid(sv)
    o, d = synth.random_rays(60, seed=36)
    o, d = o.numpy(), d.numpy()
    G = np.random.default_rng(37).normal(size=(60, 3))
    gd, gs, touched = O.render_bwd(g, o, d, G)
    md, ms = O.render_bwd_mass(g, o, d, np.abs(G))
    assert np.all(md >= np.abs(gd) * (1 - 1e-12)) and np.all(ms >= np.abs(gs) * (1 - 1e-12))
    assert np.all(md[touched == 0] == 0) and np.all(ms[touched == 0] == 0)
    # a direction where every basis value is >= 0 and dL/dC >= 0: the SH
    # terms cannot cancel, so the mass equals the gradient
    dirn = np.array([-0.6, -0.3, 0.74])
    dirn = (dirn / np.linalg.norm(dirn)).astype(np.float32)
    assert np.all(O.sh_basis(dirn.astype(np.float64)) >= 0)
    oo = (-1.5 * dirn[None, :] + np.random.default_rng(38).uniform(-0.2, 0.2, (20, 3))).astype(np.float32)
    dd = np.tile(dirn, (20, 1))
    Gp = np.abs(np.random.default_rng(39).normal(size=(20, 3)))
    _, gs2, _ = O.render_bwd(g, oo, dd, Gp)
    _, ms2 = O.render_bwd_mass(g, oo, dd, Gp)
    assert np.abs(ms2).max() > 0
    np.testing.assert_allclose(ms2, gs2, rtol=1e-12, atol=1e-300)


def test_camera_rays_match_pinhole_geometry():
    # against the independent generator (torch matmul, FP64) and geometry:
    # unit directions, the centre pixel looks at the camera's -z axis, the
    # corner pixels span the stated field of view
    poses = synth.sphere_poses(3, seed=44)
    for p in poses:
        W, H, fov = 37, 23, 45.0
        f = 0.5 * W / math.tan(0.5 * math.radians(fov))
        c2w = p.numpy().reshape(12)
        o, d = O.camera_rays(c2w, f, W, H)
        so, sd = synth.camera_rays(p, W, H, fov)
        np.testing.assert_array_equal(o, so.numpy())
        np.testing.assert_allclose(d, sd.numpy(), atol=1.2e-7, rtol=0)
        np.testing.assert_allclose(np.linalg.norm(d.astype(np.float64), axis=1), 1.0, atol=2e-7)
        fwd = -p.numpy()[:, 2]
        ang = np.degrees(np.arccos(np.clip(d.astype(np.float64) @ fwd, -1, 1)))
        half_diag = np.degrees(np.arctan(math.hypot(W - 1, H - 1) / 2 / f))
        assert abs(ang.max() - half_diag) < 1e-3


def test_gradient_mass_gate_band_adds_only_near_kink_terms():
    # with negative colours present, widening the gate band can only add
    # mass, and a zero band gives the plain mass
    sv = synth.dense_random((6, 6, 6), seed=40, ho_scale=0.6)
    g = oracle_grid(sv)
    o, d = synth.random_rays(40, seed=41)
    o, d = o.numpy(), d.numpy()
    G = np.abs(np.random.default_rng(42).normal(size=(40, 3)))
    p_d, p_s = O.render_bwd_mass(g, o, d, G)
    a_d, a_s = O.render_bwd_mass(g, o, d, G, gate_rel=0.5)
    z_d, z_s = O.render_bwd_mass(g, o, d, G, gate_rel=0.0)
    # (OpenMP accumulation order may differ between calls)
    np.testing.assert_allclose(p_s, z_s, rtol=1e-12)
    np.testing.assert_allclose(p_d, z_d, rtol=1e-12)
    assert np.all(a_s >= p_s * (1 - 1e-12)) and np.all(a_d >= p_d * (1 - 1e-12))
    assert (a_s > p_s * (1 + 1e-9)).any()
