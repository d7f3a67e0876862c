"""Pins of the FP64 oracle against things other than itself: closed forms,
special cases that reduce to library routines (scipy), invariants, brute force
and central finite differences.  CPU only.

The paper prints no image, loss or gradient value, so no pin is the paper's
own number; every pin below is a closed form or an identity the definition
implies.
"""

import numpy as np
import pytest
import scipy.linalg
import scipy.special
from scipy.spatial.transform import Rotation

import oracle

C0 = 1.0 / (2.0 * np.sqrt(np.pi))


# ----------------------------------------------------------------- helpers

def _scene(means, log_scales, quats, logit, sh, deg, viewmat, intr, wh):
    return dict(means=np.asarray(means, float), log_scales=np.asarray(log_scales, float),
                quats=np.asarray(quats, float), opacity_logit=np.asarray(logit, float),
                sh=np.asarray(sh, float), sh_degree=deg,
                viewmat=np.asarray(viewmat, float).reshape(-1, 12),
                intr=np.asarray(intr, float).reshape(-1, 4),
                wh=np.asarray(wh, np.int32).reshape(-1, 2))


def _viewmat(R, t):
    return np.concatenate([R, np.asarray(t)[:, None]], axis=1).reshape(12)


def _world_from_cam(R, t, pc):
    return R.T @ (np.asarray(pc, float) - t)


def _cs_real_sh(l, m, d):
    """Real SH with the Condon-Shortley phase, from scipy's complex SH."""
    d = np.asarray(d, float) / np.linalg.norm(d)
    theta = np.arccos(np.clip(d[2], -1, 1))
    phi = np.arctan2(d[1], d[0]) % (2 * np.pi)
    if m == 0:
        return scipy.special.sph_harm_y(l, 0, theta, phi).real
    Y = scipy.special.sph_harm_y(l, abs(m), theta, phi)
    return np.sqrt(2) * (Y.real if m > 0 else Y.imag)


def _twist_matrix(xi):
    r, f = xi[:3], xi[3:]
    return np.array([[0, -f[2], f[1], r[0]],
                     [f[2], 0, -f[0], r[1]],
                     [-f[1], f[0], 0, r[2]],
                     [0, 0, 0, 0]], float)


def _left_perturb(viewmat12, xi):
    """Exp(xi) * T by scipy's matrix exponential (not the oracle's series)."""
    T = np.eye(4)
    T[:3, :] = np.asarray(viewmat12, float).reshape(3, 4)
    return (scipy.linalg.expm(_twist_matrix(xi)) @ T)[:3, :].reshape(12)


# ----------------------------------------------------------------- projection

def test_single_isotropic_gaussian_closed_form():
    # mu = (0,0,4) in camera space, s = 0.05, o = 0.5, f = 300, c = 128
    # => cov2d = (f s / z)^2 + 0.3 = 14.3625 I; at pixel (128,128) (centre
    # 128.5) sigma = 0.5 * 0.5 / 14.3625; half extent sqrt(2 ln(127.5) 14.3625).
    rng = np.random.default_rng(0)
    R = Rotation.random(random_state=1).as_matrix()
    t = rng.normal(size=3)
    mu = _world_from_cam(R, t, [0, 0, 4])
    q = 3.0 * rng.normal(size=4)                   # not unit: the method normalises
    c_dc = 0.7
    sc = _scene(mu[:, None], np.full((3, 1), np.log(0.05)), q[:, None], [0.0],
                np.full((1, 3, 1), c_dc), 0, _viewmat(R, t), [300, 300, 128, 128], [256, 256])
    pr = oracle.project(sc)
    assert pr["valid"][0] == 1
    np.testing.assert_allclose(pr["cov2d"][0], [14.3625, 0, 14.3625], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pr["conic"][0], [1 / 14.3625, 0, 1 / 14.3625], rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(pr["mean2d"][0], [128, 128], rtol=0, atol=1e-10)
    np.testing.assert_allclose(pr["depth"][0], 4.0, rtol=1e-13)
    np.testing.assert_allclose(pr["ext"][0], [11.8009] * 2, rtol=0, atol=1e-4)
    np.testing.assert_allclose(pr["rgb"][0], [0.5 + C0 * c_dc] * 3, rtol=1e-13)
    out = oracle.render(pr, sc["wh"], pix=[128 * 256 + 128])
    sigma = 0.0174064
    assert abs(0.5 * 0.5 / 14.3625 - sigma) < 1e-7
    alpha = 0.5 * np.exp(-0.5 * 0.5 / 14.3625)
    assert abs(alpha - 0.4913721) < 1e-7
    np.testing.assert_allclose(out["rgb"][0], alpha * pr["rgb"][0], rtol=1e-13)
    np.testing.assert_allclose(out["T"][0], 1 - alpha, rtol=1e-13)


@pytest.mark.parametrize("x_over_z,clamped", [(0.2, False), (1.0, True), (-0.9, True)])
def test_axis_aligned_offaxis_closed_form(x_over_z, clamped):
    # identity camera, identity Gaussian rotation, mean (x, 0, z):
    # J = [[f/z, 0, -f tx/z], [0, f/z, 0]] with tx = x/z clamped to the padded
    # frustum [-(c/f + 0.15 W/f), (W-c)/f + 0.15 W/f].
    f, cx, W, z = 300.0, 128.0, 256, 3.0
    s = np.array([0.04, 0.07, 0.11])
    x = x_over_z * z
    sc = _scene([[x], [0.0], [z]], np.log(s)[:, None], [[1.0], [0], [0], [0]], [2.0],
                np.zeros((1, 3, 1)), 0, _viewmat(np.eye(3), np.zeros(3)),
                [f, f, cx, 128.0], [W, 256])
    pr = oracle.project(sc)
    lim = (W - cx) / f + 0.15 * W / f if x_over_z > 0 else -(cx / f + 0.15 * W / f)
    tx = lim if clamped else x / z
    assert (abs(x / z) > abs(lim)) == clamped
    a = (f / z) ** 2 * s[0] ** 2 + (f * tx / z) ** 2 * s[2] ** 2 + 0.3
    c = (f / z) ** 2 * s[1] ** 2 + 0.3
    np.testing.assert_allclose(pr["cov2d"][0], [a, 0, c], rtol=1e-12, atol=1e-12)
    np.testing.assert_allclose(pr["mean2d"][0], [f * x / z + cx, 128.0], rtol=1e-13)


def test_rotated_covariance_against_scipy_rotation():
    # On the optical axis J = [[f/z,0,0],[0,f/z,0]], so cov2d is the top-left 2x2
    # of R Rq S^2 Rq^T R^T scaled by (f/z)^2, plus 0.3 I.
    rng = np.random.default_rng(3)
    for trial in range(20):
        R = Rotation.random(random_state=trial + 10).as_matrix()
        t = rng.normal(size=3)
        z = rng.uniform(1, 8)
        q = rng.normal(size=4) * rng.uniform(0.2, 4)
        s = np.exp(rng.normal(-3, 0.5, size=3))
        mu = _world_from_cam(R, t, [0, 0, z])
        sc = _scene(mu[:, None], np.log(s)[:, None], q[:, None], [0.3], np.zeros((1, 3, 1)), 0,
                    _viewmat(R, t), [500, 400, 320, 240], [640, 480])
        pr = oracle.project(sc)
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sc = R @ Rq @ np.diag(s ** 2) @ Rq.T @ R.T
        want = np.array([500 ** 2 * Sc[0, 0] / z ** 2 + 0.3, 500 * 400 * Sc[0, 1] / z ** 2,
                         400 ** 2 * Sc[1, 1] / z ** 2 + 0.3])
        np.testing.assert_allclose(pr["cov2d"][0], want, rtol=1e-10, atol=1e-12)
        np.testing.assert_allclose(pr["depth"][0], z, rtol=1e-12)


def test_projection_jacobian_against_finite_differences():
    # cov2d - 0.3 I = J Sigma_c J^T with J the derivative of the pinhole map.
    rng = np.random.default_rng(4)
    fx, fy, cx, cy = 410.0, 380.0, 300.0, 210.0
    for trial in range(10):
        R = Rotation.random(random_state=trial + 50).as_matrix()
        t = rng.normal(size=3)
        pc = np.array([rng.uniform(-1, 1), rng.uniform(-0.8, 0.8), rng.uniform(2, 6)])
        q = rng.normal(size=4)
        s = np.exp(rng.normal(-2.5, 0.5, size=3))
        sc = _scene(_world_from_cam(R, t, pc)[:, None], np.log(s)[:, None], q[:, None], [0.0],
                    np.zeros((1, 3, 1)), 0, _viewmat(R, t), [fx, fy, cx, cy], [600, 420])
        pr = oracle.project(sc)

        def pin(p):
            return np.array([fx * p[0] / p[2] + cx, fy * p[1] / p[2] + cy])
        J = np.zeros((2, 3))
        for k in range(3):
            e = np.zeros(3); e[k] = 1e-6
            J[:, k] = (pin(pc + e) - pin(pc - e)) / 2e-6
        Rq = Rotation.from_quat([q[1], q[2], q[3], q[0]]).as_matrix()
        Sc = R @ Rq @ np.diag(s ** 2) @ Rq.T @ R.T
        C = J @ Sc @ J.T
        np.testing.assert_allclose(pr["cov2d"][0], [C[0, 0] + 0.3, C[0, 1], C[1, 1] + 0.3],
                                   rtol=1e-6, atol=1e-9)
        np.testing.assert_allclose(pr["mean2d"][0], pin(pc), rtol=1e-12)


def test_culling_rules():
    R, t = np.eye(3), np.zeros(3)
    means = np.array([[0, 0, 0.005], [0, 0, 3.0], [0, 0, 3.0]]).T
    logit = [0.0, 0.0, np.log((1 / 255) / (1 - 1 / 255)) - 1e-3]   # 3rd: o < 1/255
    sc = _scene(means, np.full((3, 3), -3.0), np.tile([[1.0], [0], [0], [0]], 3), logit,
                np.zeros((1, 3, 3)), 0, _viewmat(R, t), [300, 300, 128, 128], [256, 256])
    pr = oracle.project(sc)
    assert list(pr["valid"]) == [0, 1, 0]


# ----------------------------------------------------------------- spherical harmonics

def test_sh_low_orders_closed_form():
    d = np.array([0.3, -0.5, 0.81])
    d /= np.linalg.norm(d)
    Y = oracle.sh_basis(1, d)
    c1 = np.sqrt(3 / (4 * np.pi))
    np.testing.assert_allclose(Y, [C0, -c1 * d[1], c1 * d[2], -c1 * d[0]], rtol=1e-14)


def test_sh_matches_scipy_complex_harmonics():
    rng = np.random.default_rng(5)
    for _ in range(25):
        d = rng.normal(size=3)
        d /= np.linalg.norm(d)
        Y = oracle.sh_basis(3, d)
        for l in range(4):
            for m in range(-l, l + 1):
                assert abs(Y[l * l + l + m] - _cs_real_sh(l, m, d)) < 1e-12, (l, m)


def test_sh_orthonormal_by_quadrature():
    xg, wg = np.polynomial.legendre.leggauss(16)
    nphi = 32
    G = np.zeros((16, 16))
    for z, wz in zip(xg, wg):
        for k in range(nphi):
            ph = 2 * np.pi * k / nphi
            r = np.sqrt(1 - z * z)
            Y = oracle.sh_basis(3, [r * np.cos(ph), r * np.sin(ph), z])
            G += wz * (2 * np.pi / nphi) * np.outer(Y, Y)
    np.testing.assert_allclose(G, np.eye(16), atol=1e-12)


def test_sh_gradient_against_finite_differences():
    rng = np.random.default_rng(6)
    for _ in range(10):
        d = rng.normal(size=3)
        Y, dY = oracle.sh_basis(3, d, grad=True)
        for k in range(3):
            e = np.zeros(3); e[k] = 1e-6
            fd = (oracle.sh_basis(3, d + e) - oracle.sh_basis(3, d - e)) / 2e-6
            np.testing.assert_allclose(dY[:, k], fd, rtol=1e-6, atol=1e-8)


def test_colour_uses_view_direction_from_camera_centre():
    # Gaussian on the optical axis: the world view direction is the camera's
    # forward axis, the third row of R.
    rng = np.random.default_rng(7)
    R = Rotation.random(random_state=77).as_matrix()
    t = rng.normal(size=3)
    sh = rng.normal(0, 0.3, size=(16, 3, 1))
    sc = _scene(_world_from_cam(R, t, [0, 0, 2.5])[:, None], np.full((3, 1), -3.0),
                [[1.0], [0], [0], [0]], [0.0], sh, 3, _viewmat(R, t), [300, 300, 128, 128],
                [256, 256])
    pr = oracle.project(sc)
    d = R[2]
    want = [max(0.0, 0.5 + sum(_cs_real_sh(l, m, d) * sh[l * l + l + m, ch, 0]
                                for l in range(4) for m in range(-l, l + 1))) for ch in range(3)]
    np.testing.assert_allclose(pr["rgb"][0], want, rtol=1e-11, atol=1e-13)
    sh2 = sh.copy()
    sh2[0] = -10.0                             # colour clamps at 0
    pr2 = oracle.project(dict(sc, sh=sh2))
    np.testing.assert_array_equal(pr2["rgb"][0], [0, 0, 0])


# ----------------------------------------------------------------- compositing

def _stack_proj(n, alpha, rgb=(0.2, 0.6, 0.9), px=(10.5, 7.5)):
    """n splats centred on one pixel with opacity alpha (sigma = 0 there)."""
    return dict(valid=np.ones(n, np.int32), depth=np.linspace(1, 2, n),
                mean2d=np.tile(px, (n, 1)), conic=np.tile([0.5, 0.0, 0.5], (n, 1)),
                opacity=np.full(n, alpha), rgb=np.tile(rgb, (n, 1)))


@pytest.mark.parametrize("alpha,count", [(0.5, 13), (0.3, 25), (0.7, 7)])
def test_early_termination_closed_form(alpha, count):
    # (1-alpha)^count >= 1e-4 > (1-alpha)^(count+1): exactly `count` splats blend.
    assert (1 - alpha) ** count >= 1e-4 > (1 - alpha) ** (count + 1)
    n = 40
    pr = _stack_proj(n, alpha)
    wh = np.array([[32, 16]], np.int32)
    out = oracle.render(pr, wh, pix=[7 * 32 + 10])
    assert out["ncontrib"][0] == count
    np.testing.assert_allclose(out["T"][0], (1 - alpha) ** count, rtol=1e-13)
    np.testing.assert_allclose(out["rgb"][0], np.array([0.2, 0.6, 0.9]) * (1 - (1 - alpha) ** count),
                               rtol=1e-12)
    assert out["T"][0] >= 1e-4


@pytest.mark.parametrize("factor,included", [(1 - 1e-3, False), (1 + 1e-3, True)])
def test_alpha_gate(factor, included):
    # o exp(-sigma) = factor / 255 at the pixel
    o = 0.6
    sigma = np.log(o * 255 / factor)
    A = 0.05
    dx = np.sqrt(2 * sigma / A)
    pr = dict(valid=np.ones(1, np.int32), depth=np.ones(1), mean2d=np.array([[10.5 + dx, 7.5]]),
              conic=np.array([[A, 0.0, 0.3]]), opacity=np.array([o]), rgb=np.array([[1.0, 1, 1]]))
    out = oracle.render(pr, np.array([[64, 16]], np.int32), pix=[7 * 64 + 10])
    assert out["ngate"][0] == int(included)
    if included:
        np.testing.assert_allclose(out["rgb"][0], [factor / 255] * 3, rtol=1e-9)
    else:
        np.testing.assert_array_equal(out["rgb"][0], [0, 0, 0])


def _small_scene(seed, W=40, H=30, N=60, deg=3, unit_quats=False):
    import scenegen
    return scenegen.frustum_scene(seed, W, H, 0.9 * W, 0.9 * W, N, deg, -2.2, 0.4,
                                  sh_sd=None if deg == 0 else 0.25, unit_quats=unit_quats)


def test_partition_of_unity_and_transmittance_bounds():
    sc = _small_scene(11, N=300, deg=0)
    pr = oracle.project(sc)
    pr1 = dict(pr, rgb=np.ones_like(pr["rgb"]))
    out = oracle.render(pr1, sc["wh"])
    np.testing.assert_allclose(out["rgb"][:, 0], 1 - out["T"], atol=1e-13)
    assert np.all(out["T"] >= 1e-4) and np.all(out["T"] <= 1)
    assert out["ncontrib"].max() > 5


def test_result_independent_of_gaussian_order():
    sc = _small_scene(12, N=200, deg=3)
    perm = np.random.default_rng(0).permutation(200)
    sc2 = dict(sc)
    for k in ("means", "log_scales", "quats"):
        sc2[k] = sc[k][:, perm]
    sc2["opacity_logit"] = sc["opacity_logit"][perm]
    sc2["sh"] = sc["sh"][:, :, perm]
    a = oracle.render_fwd_bwd(sc)
    b = oracle.render_fwd_bwd(sc2)
    np.testing.assert_allclose(a["rgb"], b["rgb"], atol=1e-14)


# ----------------------------------------------------------------- gradients

def _loss(sc, w, viewmat=None):
    out = oracle.render_fwd_bwd(sc, viewmat=viewmat)
    return float(np.sum(out["rgb"] * w)), out


def _clamp_state(out):
    """Everything that selects a branch: gate counts, contributor counts, the
    colour clamp and the depth order."""
    return (out["ncontrib"].copy(), out["ngate"].copy(), (out["proj"]["rgb"] == 0).copy(),
            np.argsort(out["proj"]["depth"], kind="stable"))


def _same_state(a, b):
    return all(np.array_equal(x, y) for x, y in zip(a, b))


def test_parameter_gradients_against_central_differences():
    # 60 Gaussians in a 40x30 view, SH degree 3, non-unit quaternions; a few
    # large off-screen Gaussians exercise the clamped Jacobian.
    sc = _small_scene(13, N=60, deg=3)
    sc = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype == np.float32 else v)
          for k, v in sc.items()}
    # push 4 Gaussians outside the padded frustum but big enough to reach the image
    R = sc["viewmat"][0].reshape(3, 4)[:, :3]
    t = sc["viewmat"][0].reshape(3, 4)[:, 3]
    for j, pc in enumerate([[3.2, 0.1, 2.03], [-3.0, 0.2, 2.21], [0.1, 2.6, 2.12], [0.0, -2.5, 1.97]]):
        sc["means"][:, j] = _world_from_cam(R, t, pc)
        sc["log_scales"][:, j] = np.log([0.9, 0.9, 0.9])
    w = np.random.default_rng(1).normal(size=(40 * 30, 3))
    L0, base = _loss(sc, w)
    st0 = _clamp_state(base)
    an = oracle.render_fwd_bwd(sc, v_rgb=w)["grads"]
    n_checked = 0
    for key in ("means", "log_scales", "quats", "opacity_logit", "sh"):
        arr = sc[key]
        flat = arr.reshape(-1)
        fd = np.zeros_like(flat)
        ok = np.zeros(flat.shape, bool)
        for i in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            Lp, op = _loss(sc, w)
            flat[i] = old - h
            Lm, om = _loss(sc, w)
            flat[i] = old
            if _same_state(st0, _clamp_state(op)) and _same_state(st0, _clamp_state(om)):
                fd[i] = (Lp - Lm) / (2 * h)
                ok[i] = True
        a = an[key].reshape(-1)
        scale = np.max(np.abs(a)) + 1e-30
        err = np.abs(a[ok] - fd[ok])
        assert ok.mean() > 0.95, key
        assert np.max(err) <= 1e-6 * scale + 1e-9, (key, np.max(err), scale)
        n_checked += ok.sum()
    assert n_checked > 3000


def test_pose_twist_gradient_against_central_differences():
    for deg, seed in ((0, 21), (3, 22)):
        sc = _small_scene(seed, N=80, deg=deg)
        w = np.random.default_rng(seed).normal(size=(40 * 30, 3))
        an = oracle.render_fwd_bwd(sc, v_rgb=w)["grads"]["twist"][0]
        L0, base = _loss(sc, w)
        st0 = _clamp_state(base)
        for k in range(6):
            xi = np.zeros(6)
            xi[k] = 1e-6
            Lp, op = _loss(sc, w, viewmat=_left_perturb(sc["viewmat"][0], xi)[None])
            Lm, om = _loss(sc, w, viewmat=_left_perturb(sc["viewmat"][0], -xi)[None])
            assert _same_state(st0, _clamp_state(op)) and _same_state(st0, _clamp_state(om))
            fd = (Lp - Lm) / 2e-6
            assert abs(fd - an[k]) <= 1e-6 * np.max(np.abs(an)) + 1e-9, (deg, k, fd, an[k])


def test_twist_gauge_identities():
    # Moving the camera by rho equals moving every Gaussian by R^T rho, so
    # g_rho = R sum_g dL/dmu_g (any SH degree).  With SH degree 0, turning the
    # camera by phi equals turning every Gaussian about the camera centre by
    # omega = R^T phi, so g_phi = R sum_g [(mu_g - c) x dL/dmu_g + dL/domega_g].
    for deg in (0, 3):
        sc = dict(_small_scene(30 + deg, N=120, deg=deg, unit_quats=True))
        # the identities need an exactly orthonormal R (the float32 one is not)
        M = sc["viewmat"][0].reshape(3, 4).astype(float)
        U, _, Vt = np.linalg.svd(M[:, :3])
        sc["viewmat"] = _viewmat(U @ Vt, M[:, 3])[None]
        sc["quats"] = sc["quats"].astype(float) / np.linalg.norm(sc["quats"].astype(float), axis=0)
        w = np.random.default_rng(deg).normal(size=(40 * 30, 3))
        g = oracle.render_fwd_bwd(sc, v_rgb=w)["grads"]
        M = sc["viewmat"][0].reshape(3, 4).astype(float)
        R, t = M[:, :3], M[:, 3]
        vmu = g["means"]                                # [3,N]
        np.testing.assert_allclose(g["twist"][0, :3], R @ vmu.sum(axis=1),
                                   rtol=1e-9, atol=1e-12 * np.abs(g["twist"]).max())
        if deg == 0:
            c = -R.T @ t
            mu = sc["means"].astype(float)
            q = sc["quats"].astype(float)
            vq = g["quats"]
            # quaternion left-multiplied by (1, omega/2):  dq = 0.5 (0,omega) (x) q
            vomega = 0.5 * (-vq[0] * q[1:] + q[0] * vq[1:] + np.cross(q[1:].T, vq[1:].T).T)
            tot = np.cross((mu - c[:, None]).T, vmu.T).sum(axis=0) + vomega.sum(axis=1)
            np.testing.assert_allclose(g["twist"][0, 3:], R @ tot, rtol=1e-9,
                                       atol=1e-12 * np.abs(g["twist"]).max())


# ----------------------------------------------------------------- track term

def _track_setup(seed=40, M=60, Pt=20, ncam=3):
    rng = np.random.default_rng(seed)
    vms, intr = [], []
    for i in range(ncam):
        R = Rotation.random(random_state=seed + i).as_matrix()
        vms.append(_viewmat(R, rng.normal(size=3)))
        intr.append([rng.uniform(200, 400), rng.uniform(200, 400), 160.0, 120.0])
    vms, intr = np.array(vms), np.array(intr)
    X = np.zeros((Pt, 3))
    cam = np.sort(rng.integers(0, ncam, size=M))
    pt = rng.integers(0, Pt, size=M)
    for k in range(Pt):
        i = cam[np.nonzero(pt == k)[0][0]] if np.any(pt == k) else 0
        M3 = vms[i].reshape(3, 4)
        X[k] = _world_from_cam(M3[:, :3], M3[:, 3], [rng.uniform(-1, 1), rng.uniform(-1, 1), rng.uniform(3, 6)])
    xy = np.zeros((M, 2))
    for o in range(M):
        M3 = vms[cam[o]].reshape(3, 4)
        p = M3[:, :3] @ X[pt[o]] + M3[:, 3]
        f = intr[cam[o]]
        xy[o] = [f[0] * p[0] / p[2] + f[2], f[1] * p[1] / p[2] + f[3]]
    xy += rng.normal(0, 1.5, size=(M, 2))            # mix of Huber inliers and outliers
    return X, vms, intr, cam.astype(np.int32), pt.astype(np.int32), xy


def test_track_optical_axis_closed_form():
    vm = _viewmat(np.eye(3), np.zeros(3))
    for dxy, rho in (((3.0, 4.0), 2 * 5 - 1), ((0.3, 0.4), 0.25)):
        out = oracle.track(np.array([[0, 0, 5.0]]), vm[None], np.array([[300, 300, 100, 80.0]]),
                           np.array([0], np.int32), np.array([0], np.int32),
                           np.array([[100 + dxy[0], 80 + dxy[1]]]), delta=1.0, lam=0.5)
        np.testing.assert_allclose(out["residual"][0], [-dxy[0], -dxy[1]], atol=1e-12)
        np.testing.assert_allclose(out["loss"], 0.5 * rho, rtol=1e-12)


def test_huber_continuity_at_threshold():
    vm = _viewmat(np.eye(3), np.zeros(3))
    vals, slopes = [], []
    for r in (2.0 - 1e-9, 2.0 + 1e-9):            # delta = 2: |r| = delta
        out = oracle.track(np.array([[0, 0, 5.0]]), vm[None], np.array([[300, 300, 100, 80.0]]),
                           np.array([0], np.int32), np.array([0], np.int32),
                           np.array([[100 + r, 80.0]]), delta=2.0, lam=1.0)
        vals.append(out["loss"])
        slopes.append(out["v_X"][0, 0])
    assert abs(vals[0] - vals[1]) < 1e-7
    assert abs(slopes[0] - slopes[1]) < 1e-6 * abs(slopes[0])


def test_track_gradients_and_jacobians_against_central_differences():
    X, vms, intr, cam, pt, xy = _track_setup()
    out = oracle.track(X, vms, intr, cam, pt, xy, delta=1.0, lam=1e-4)
    assert 0 < np.mean(np.sum(out["residual"] ** 2, 1) <= 1) < 1     # both branches
    h = 1e-6
    for k in range(X.shape[0]):
        for e in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[k, e] += h
            Xm[k, e] -= h
            fd = (oracle.track(Xp, vms, intr, cam, pt, xy)["loss"] -
                  oracle.track(Xm, vms, intr, cam, pt, xy)["loss"]) / (2 * h)
            assert abs(fd - out["v_X"][k, e]) <= 1e-6 * np.abs(out["v_X"]).max()
    for i in range(vms.shape[0]):
        for k in range(6):
            xi = np.zeros(6); xi[k] = h
            vp, vm_ = vms.copy(), vms.copy()
            vp[i] = _left_perturb(vms[i], xi)
            vm_[i] = _left_perturb(vms[i], -xi)
            fd = (oracle.track(X, vp, intr, cam, pt, xy)["loss"] -
                  oracle.track(X, vm_, intr, cam, pt, xy)["loss"]) / (2 * h)
            assert abs(fd - out["v_twist"][i, k]) <= 1e-6 * np.abs(out["v_twist"]).max()
    # Jacobian blocks of the residual
    for o in range(0, len(cam), 7):
        i = cam[o]
        for k in range(6):
            xi = np.zeros(6); xi[k] = h
            vp, vm_ = vms.copy(), vms.copy()
            vp[i] = _left_perturb(vms[i], xi)
            vm_[i] = _left_perturb(vms[i], -xi)
            fd = (oracle.track(X, vp, intr, cam, pt, xy)["residual"][o] -
                  oracle.track(X, vm_, intr, cam, pt, xy)["residual"][o]) / (2 * h)
            np.testing.assert_allclose(out["J_pose"][o][:, k], fd, rtol=1e-6, atol=1e-6)
        for e in range(3):
            Xp, Xm = X.copy(), X.copy()
            Xp[pt[o], e] += h
            Xm[pt[o], e] -= h
            fd = (oracle.track(Xp, vms, intr, cam, pt, xy)["residual"][o] -
                  oracle.track(Xm, vms, intr, cam, pt, xy)["residual"][o]) / (2 * h)
            np.testing.assert_allclose(out["J_X"][o][:, e], fd, rtol=1e-6, atol=1e-6)


def test_track_single_camera_gauge_and_masking():
    X, vms, intr, cam, pt, xy = _track_setup(seed=41, ncam=1)
    out = oracle.track(X, vms, intr, cam, pt, xy, lam=1.0)
    R = vms[0].reshape(3, 4)[:, :3]
    np.testing.assert_allclose(out["v_X"].sum(axis=0), R.T @ out["v_twist"][0, :3], rtol=1e-10,
                               atol=1e-12)
    # a point behind the camera is masked: no loss, no gradient, counted
    X2 = X.copy()
    M3 = vms[0].reshape(3, 4)
    X2[pt[0]] = _world_from_cam(M3[:, :3], M3[:, 3], [0.1, 0.1, -2.0])
    out2 = oracle.track(X2, vms, intr, cam, pt, xy, lam=1.0)
    masked = out2["masked"].astype(bool)
    assert masked.sum() == np.sum(pt == pt[0])
    np.testing.assert_array_equal(out2["v_X"][pt[0]], 0)


# ----------------------------------------------------------------- SE(3) and Adam

def test_se3_exp_against_scipy():
    rng = np.random.default_rng(50)
    for _ in range(10):
        xi = rng.normal(size=6) * rng.uniform(0.001, 2)
        base = np.concatenate([Rotation.random(random_state=int(rng.integers(1e6))).as_matrix(),
                               rng.normal(size=(3, 1))], axis=1).reshape(12)
        out = oracle.se3_exp_compose(xi, base)[0]
        np.testing.assert_allclose(out, _left_perturb(base, xi), rtol=1e-12, atol=1e-12)
        # rotation part is Rodrigues' rotation of the axis-angle phi
        Rr = Rotation.from_rotvec(xi[3:]).as_matrix() @ base.reshape(3, 4)[:, :3]
        np.testing.assert_allclose(out.reshape(3, 4)[:, :3], Rr, atol=1e-12)


def test_se3_left_jacobian_against_finite_differences():
    # Exp(xi + d) = Exp(J_l(xi) d) Exp(xi) to first order, so the gradient of a
    # function of Exp(xi + d) T0 w.r.t. d is J_l(xi)^T times its gradient under a
    # left perturbation at Exp(xi) T0.
    rng = np.random.default_rng(51)
    for _ in range(8):
        xi = rng.normal(size=6) * rng.uniform(0.01, 1.5)
        T0 = np.concatenate([Rotation.random(random_state=int(rng.integers(1e6))).as_matrix(),
                             rng.normal(size=(3, 1))], axis=1).reshape(12)
        Wt = rng.normal(size=12)

        def f(T):
            return float(Wt @ T)
        T = _left_perturb(T0, xi)
        h = 1e-6
        g = np.array([(f(_left_perturb(T, h * e)) - f(_left_perturb(T, -h * e))) / (2 * h)
                      for e in np.eye(6)])
        gd = np.array([(f(_left_perturb(T0, xi + h * e)) - f(_left_perturb(T0, xi - h * e))) / (2 * h)
                       for e in np.eye(6)])
        np.testing.assert_allclose(oracle.se3_jl_transpose(xi, g)[0], gd, rtol=1e-6, atol=1e-7)


def test_adam_first_step_and_constant_gradient():
    rng = np.random.default_rng(52)
    g = rng.normal(size=100)
    p = rng.normal(size=100)
    p0 = p.copy()
    m = np.zeros(100)
    v = np.zeros(100)
    lr, eps = 1e-3, 1e-8
    oracle.adam(p, g, m, v, lr, eps=eps, step=1)
    # first step: m_hat = g, v_hat = g^2
    np.testing.assert_allclose(p, p0 - lr * g / (np.abs(g) + eps), rtol=1e-12)
    # a constant gradient keeps m_hat = g, v_hat = g^2: every step moves the same
    for step in range(2, 12):
        before = p.copy()
        oracle.adam(p, g, m, v, lr, eps=eps, step=step)
        np.testing.assert_allclose(before - p, lr * g / (np.abs(g) + eps), rtol=1e-9)


# ----------------------------------------------------------------- tile lists

def test_tile_membership_against_dense_sampling():
    # A pair belongs to a tile iff some point of one of the tile's quadrant
    # rectangles (spanned by the quadrant's pixel centres) has alpha >= 1/255.
    # Brute force: sample every quadrant rectangle densely.
    rng = np.random.default_rng(60)
    W, H, N = 70, 45, 40
    mean2d = np.stack([rng.uniform(-10, W + 10, N), rng.uniform(-10, H + 10, N)], 1)
    cov = []
    for _ in range(N):
        A = rng.normal(size=(2, 2)) * rng.uniform(1, 6)
        cov.append(A @ A.T + 0.3 * np.eye(2))
    conic = np.array([[c[1, 1], -c[0, 1], c[0, 0]] / np.linalg.det(c) for c in cov])
    opac = rng.uniform(0.02, 0.99, N)
    depth = rng.uniform(1, 5, N).astype(np.float32)
    valid = np.ones(N, np.int32)
    ranges, ids, masks = oracle.bin_sort(np.array([[W, H]]), (16, 16), valid, mean2d, conic, opac,
                                         depth, with_masks=True)
    gx = (W + 15) // 16
    for t in range(ranges.shape[0]):
        tx, ty = t % gx, t // gx
        members = dict(zip(ids[ranges[t, 0]:ranges[t, 1]].tolist(),
                           masks[ranges[t, 0]:ranges[t, 1]].tolist()))
        for g in range(N):
            want = 0
            loose = 0
            for q in range(4):
                xs, ys = tx * 16 + (q & 1) * 8, ty * 16 + (q >> 1) * 8
                if xs >= W or ys >= H:
                    continue
                xq = np.linspace(xs + 0.5, min(xs + 8, W) - 0.5, 41)
                yq = np.linspace(ys + 0.5, min(ys + 8, H) - 0.5, 41)
                X, Y = np.meshgrid(xq, yq)
                dx, dy = mean2d[g, 0] - X, mean2d[g, 1] - Y
                sg = 0.5 * (conic[g, 0] * dx * dx + conic[g, 2] * dy * dy) + conic[g, 1] * dx * dy
                thr = np.log(opac[g] * 255)
                if sg.min() < thr - 1e-6:
                    want |= 1 << q
                if sg.min() < thr + 0.05 * max(1.0, thr):   # the grid is coarse
                    loose |= 1 << q
            m = members.get(g, 0)
            assert (m & want) == want, (t, g, m, want)
            assert (m & ~loose) == 0, (t, g, m, loose)
        # order: float32 depth bits, then index
        lst = ids[ranges[t, 0]:ranges[t, 1]]
        keys = [(depth[i].view(np.uint32), i) for i in lst]
        assert keys == sorted(keys)


# ----------------------------------------------------------------- order, clamp, background

def _one_pixel(pr, W=32, H=16, px=(10, 7), **kw):
    wh = np.array([[W, H]], np.int32)
    return oracle.render(pr, wh, pix=[px[1] * W + px[0]], **kw)


def _splats(depth, mean2d, conic, opacity, rgb):
    n = len(depth)
    return dict(valid=np.ones(n, np.int32), depth=np.asarray(depth, float),
                mean2d=np.asarray(mean2d, float).reshape(n, 2),
                conic=np.asarray(conic, float).reshape(n, 3),
                opacity=np.asarray(opacity, float), rgb=np.asarray(rgb, float).reshape(n, 3))


def test_compositing_order_is_float32_depth_then_index():
    # Splats 0 and 1 have FP64 depths 1e-8 apart (a twentieth of a float32 ulp
    # at 3): both round to 3.0f, so index 0 composites first although it is
    # farther.  Splats 2 and 3 are one float32 ulp apart: depth decides.
    c0, c1 = np.array([1.0, 0.0, 0.0]), np.array([0.0, 0.0, 1.0])
    a0, a1 = 0.6, 0.3
    up = float(np.nextafter(np.float32(3.0), np.float32(4.0)))
    for d0, d1, first in ((3.0 + 1e-8, 3.0, 0), (up, 3.0, 1)):
        assert (np.float32(d0) == np.float32(d1)) == (first == 0)
        pr = _splats([d0, d1], [[10.5, 7.5]] * 2, [[0.5, 0, 0.5]] * 2, [a0, a1], [c0, c1])
        out = _one_pixel(pr)
        if first == 0:
            want = c0 * a0 + c1 * a1 * (1 - a0)
        else:
            want = c1 * a1 + c0 * a0 * (1 - a1)
        np.testing.assert_allclose(out["rgb"][0], want, rtol=1e-14)


def test_depth_order_ambiguity_only_near_a_rounding_midpoint():
    # equal float32 depths, FP64 depths far from a rounding midpoint: the
    # order (by index) is certain; the same pair with one depth 1e-15 relative
    # from a midpoint is flagged
    f = np.float32(3.0)
    up = np.nextafter(f, np.float32(4.0))
    mid = 0.5 * (float(f) + float(up))
    pr = _splats([3.0 + 1e-8, 3.0], [[10.5, 7.5]] * 2, [[0.5, 0, 0.5]] * 2, [0.6, 0.3],
                 [[1, 0, 0], [0, 0, 1]])
    assert not _one_pixel(pr)["ambiguous"][0]
    pr["depth"][0] = mid * (1 + 1e-15)
    assert _one_pixel(pr)["ambiguous"][0]
    # far apart in float32: never ambiguous
    pr["depth"][1] = 2.0
    assert not _one_pixel(pr)["ambiguous"][0]


def test_alpha_clamp_closed_form():
    # o = 0.995 at the splat's own centre: alpha = min(0.99, 0.995) = 0.99
    c = np.array([0.2, 0.5, 0.9])
    pr = _splats([2.0], [[10.5, 7.5]], [[0.5, 0.0, 0.5]], [0.995], [c])
    v = np.array([[0.3, -0.7, 1.1]])
    out = _one_pixel(pr, v_rgb=v)
    np.testing.assert_allclose(out["rgb"][0], 0.99 * c, rtol=1e-15)
    np.testing.assert_allclose(out["T"][0], 0.01, rtol=1e-13)
    assert out["nclamp"][0] == 1
    # off-centre with sigma = 0.002 the raw alpha 0.995 e^-0.002 = 0.99301 is
    # still clamped: no gradient reaches the opacity or the geometry, the
    # colour gets alpha T = 0.99
    dx = np.sqrt(2 * 0.002 / 0.5)
    pr = _splats([2.0], [[10.5 + dx, 7.5]], [[0.5, 0.0, 0.5]], [0.995], [c])
    out = _one_pixel(pr, v_rgb=v)
    g = out["v2d"][0]
    np.testing.assert_array_equal(g[:6], 0.0)
    np.testing.assert_allclose(g[6:], 0.99 * v[0], rtol=1e-14)
    np.testing.assert_allclose(out["rgb"][0], 0.99 * c, rtol=1e-15)
    # below the clamp (o = 0.985): alpha = o e^-sigma and d alpha / d o = e^-sigma
    pr = _splats([2.0], [[10.5 + dx, 7.5]], [[0.5, 0.0, 0.5]], [0.985], [c])
    out = _one_pixel(pr, v_rgb=v)
    a = 0.985 * np.exp(-0.002)
    np.testing.assert_allclose(out["rgb"][0], a * c, rtol=1e-14)
    np.testing.assert_allclose(out["v2d"][0, 5], np.exp(-0.002) * float(v[0] @ c), rtol=1e-13)
    assert out["nclamp"][0] == 0


def test_background_closed_form():
    # two splats in front of a background: C = c0 a0 + c1 a1 (1 - a0)
    # + (1 - a0)(1 - a1) bg, and dC/da0 = c0 - c1 a1 - (1 - a1) bg
    bg = np.array([0.25, 0.5, 0.75])
    c0, c1 = np.array([0.9, 0.1, 0.3]), np.array([0.2, 0.8, 0.4])
    o0, o1, sig = 0.7, 0.45, 0.1
    dx = np.sqrt(2 * sig / 0.5)
    pr = _splats([1.0, 2.0], [[10.5 + dx, 7.5], [10.5, 7.5]], [[0.5, 0, 0.5]] * 2, [o0, o1],
                 [c0, c1])
    v = np.array([[0.4, -1.3, 0.8]])
    out = _one_pixel(pr, bg=bg, v_rgb=v)
    a0, a1 = o0 * np.exp(-sig), o1
    want = c0 * a0 + c1 * a1 * (1 - a0) + (1 - a0) * (1 - a1) * bg
    np.testing.assert_allclose(out["rgb"][0], want, rtol=1e-14)
    dC_da0 = c0 - c1 * a1 - (1 - a1) * bg
    np.testing.assert_allclose(out["v2d"][0, 5], np.exp(-sig) * float(v[0] @ dC_da0), rtol=1e-12)
    dC_da1 = (1 - a0) * (c1 - bg)
    np.testing.assert_allclose(out["v2d"][1, 5], float(v[0] @ dC_da1), rtol=1e-12)
    # a pixel no splat reaches shows the background with T = 1
    out = oracle.render(pr, np.array([[32, 16]], np.int32), pix=[15 * 32 + 31], bg=bg)
    np.testing.assert_array_equal(out["rgb"][0], bg)
    assert out["T"][0] == 1.0


def _clamp_state2(out):
    return _clamp_state(out) + (out["nclamp"].copy(),)


def test_gradients_with_background_and_clamped_splats_against_central_differences():
    # a background colour and a fifth of the Gaussians above the 0.99 opacity
    # clamp (logit 7..9, large): the clamped hits pass no opacity or geometry
    # gradient, the background enters dC/dalpha through T_final bg
    sc = _small_scene(17, N=50, deg=1)
    sc = {k: (v.astype(np.float64) if isinstance(v, np.ndarray) and v.dtype == np.float32 else v)
          for k, v in sc.items()}
    rng = np.random.default_rng(3)
    hi = rng.choice(50, 10, replace=False)
    sc["opacity_logit"][hi] = rng.uniform(7.0, 9.0, size=10)
    sc["log_scales"][:, hi] = np.log(rng.uniform(0.6, 1.0, size=(3, 10)))
    bg = np.array([0.3, 0.6, 0.9])
    w = rng.normal(size=(40 * 30, 3))

    def loss(viewmat=None):
        out = oracle.render_fwd_bwd(sc, bg=bg, viewmat=viewmat)
        return float(np.sum(out["rgb"] * w)), out

    L0, base = loss()
    assert base["nclamp"].sum() > 20
    st0 = _clamp_state2(base)
    an = oracle.render_fwd_bwd(sc, v_rgb=w, bg=bg)["grads"]
    for key in ("means", "log_scales", "quats", "opacity_logit"):
        flat = sc[key].reshape(-1)
        a = an[key].reshape(-1)
        errs, n_ok = [], 0
        for i in range(flat.size):
            h = 1e-6 * max(1.0, abs(flat[i]))
            old = flat[i]
            flat[i] = old + h
            Lp, op = loss()
            flat[i] = old - h
            Lm, om = loss()
            flat[i] = old
            if _same_state(st0, _clamp_state2(op)) and _same_state(st0, _clamp_state2(om)):
                errs.append(abs(a[i] - (Lp - Lm) / (2 * h)))
                n_ok += 1
        assert n_ok > 0.95 * flat.size, key
        assert max(errs) <= 1e-6 * np.max(np.abs(a)) + 1e-9, (key, max(errs))
    for k in range(6):
        xi = np.zeros(6)
        xi[k] = 1e-6
        Lp, op = loss(_left_perturb(sc["viewmat"][0], xi)[None])
        Lm, om = loss(_left_perturb(sc["viewmat"][0], -xi)[None])
        assert _same_state(st0, _clamp_state2(op)) and _same_state(st0, _clamp_state2(om))
        assert abs((Lp - Lm) / 2e-6 - an["twist"][0, k]) <= 1e-6 * np.abs(an["twist"]).max() + 1e-9


# ----------------------------------------------------------------- photometric terms

def test_l1_closed_form_view_weighting_and_ties():
    # two views of different sizes, |d| = 0.1 on the first and 0.3 on the
    # second: the mean over views is 0.2 (pooling all pixels would give 0.277)
    wh = np.array([[8, 5], [20, 11]], np.int32)
    P0, P1 = 40, 220
    rng = np.random.default_rng(2)
    t = rng.uniform(0.3, 0.7, size=(P0 + P1, 3))
    s = np.where(rng.uniform(size=t.shape) < 0.5, -1.0, 1.0)
    x = t + s * np.concatenate([np.full((P0, 3), 0.1), np.full((P1, 3), 0.3)])
    loss, v = oracle.l1(x, t, wh)
    assert abs(loss - 0.2) < 1e-14
    np.testing.assert_allclose(v[:P0], s[:P0] / (3 * P0 * 2), rtol=1e-15)
    np.testing.assert_allclose(v[P0:], s[P0:] / (3 * P1 * 2), rtol=1e-15)
    x[:7] = t[:7]                                   # exact ties: sign(0) = 0
    loss, v = oracle.l1(x, t, wh)
    np.testing.assert_array_equal(v[:7], 0.0)
    # central differences away from ties
    h = 1e-7
    for i in rng.choice(x.size, 20, replace=False):
        xp, xm = x.copy().reshape(-1), x.copy().reshape(-1)
        if xp[i] == t.reshape(-1)[i]:
            continue
        xp[i] += h
        xm[i] -= h
        fd = (oracle.l1(xp.reshape(x.shape), t, wh)[0] - oracle.l1(xm.reshape(x.shape), t, wh)[0]) / (2 * h)
        assert abs(fd - v.reshape(-1)[i]) <= 1e-6 * abs(v.reshape(-1)[i])


def _gauss_window_1d(win=11, sigma=1.5):
    i = np.arange(win) - win // 2
    g = np.exp(-i ** 2 / (2 * sigma ** 2))
    return g / g.sum()


def _ssim_scalar(mx, my, sxx, syy, sxy, c1=oracle.SSIM_C1, c2=oracle.SSIM_C2):
    return (2 * mx * my + c1) * (2 * sxy + c2) / ((mx ** 2 + my ** 2 + c1) * (sxx + syy + c2))


def test_ssim_of_an_image_with_itself_is_one_with_zero_gradient():
    rng = np.random.default_rng(5)
    wh = np.array([[23, 17], [9, 6]], np.int32)
    x = rng.uniform(size=(23 * 17 + 54, 3))
    s, v, m = oracle.ssim(x, x, wh, ssim_map=True)
    assert abs(s - 1) < 1e-14
    np.testing.assert_allclose(m, 1.0, atol=1e-14)
    np.testing.assert_allclose(v, 0.0, atol=1e-14)
    y = rng.uniform(size=x.shape)
    assert abs(oracle.ssim(x, y, wh, grad=False)[0] - oracle.ssim(y, x, wh, grad=False)[0]) < 1e-15


def test_ssim_constant_images_closed_form_interior_and_border():
    # constants a, b with zeros beyond the border: at a pixel whose window keeps
    # mass m inside the image, mu = a m, E_xx = a^2 m, so s_xx = a^2 m (1 - m)
    # and s_xy = a b m (1 - m); inside (m = 1) S = (2ab + c1) / (a^2 + b^2 + c1)
    W, H = 30, 24
    a, b = 0.62, 0.35
    x = np.full((W * H, 3), a)
    y = np.full((W * H, 3), b)
    _, _, m = oracle.ssim(x, y, np.array([[W, H]], np.int32), grad=False, ssim_map=True)
    m = m[:, 0].reshape(H, W)
    g = _gauss_window_1d()
    for (px, py) in ((15, 12), (0, 0), (3, 0), (29, 10), (7, 22)):
        mx = sum(g[i + 5] for i in range(-5, 6) if 0 <= px + i < W)
        my = sum(g[j + 5] for j in range(-5, 6) if 0 <= py + j < H)
        mass = mx * my
        want = _ssim_scalar(a * mass, b * mass, a * a * mass * (1 - mass), b * b * mass * (1 - mass),
                            a * b * mass * (1 - mass))
        # (E_xx - mu^2 cancels: rounding ~1e-16 against c2 ~1e-3)
        assert abs(m[py, px] - want) <= 1e-10, (px, py, m[py, px], want)
    assert abs(m[12, 15] - (2 * a * b + oracle.SSIM_C1) / (a * a + b * b + oracle.SSIM_C1)) < 1e-10


def test_ssim_ramp_closed_form():
    # x a ramp along u with slope s, y = k x + c: inside the image the window
    # (symmetric, unit mass) gives mu_x = x(p), s_xx = s^2 var_w with var_w the
    # window's second moment, s_xy = k s_xx, s_yy = k^2 s_xx
    W, H = 40, 30
    s_, k, c = 0.013, -0.7, 0.8
    u = np.tile(np.arange(W), H).astype(float)
    x = np.repeat((0.1 + s_ * u)[:, None], 3, axis=1)
    y = k * x + c
    _, _, m = oracle.ssim(x, y, np.array([[W, H]], np.int32), grad=False, ssim_map=True)
    g = _gauss_window_1d()
    var_w = float(np.sum(g * (np.arange(11) - 5.0) ** 2))
    for (px, py) in ((5, 5), (20, 15), (34, 24)):
        mu = 0.1 + s_ * px
        sxx = s_ * s_ * var_w
        want = _ssim_scalar(mu, k * mu + c, sxx, k * k * sxx, k * sxx)
        got = m.reshape(H, W, 3)[py, px]
        np.testing.assert_allclose(got, want, rtol=1e-12)


def test_ssim_gradient_against_central_differences():
    rng = np.random.default_rng(6)
    wh = np.array([[14, 9], [7, 5]], np.int32)    # one view smaller than the window
    P = 14 * 9 + 35
    x = rng.uniform(size=(P, 3))
    y = np.clip(x + rng.normal(0, 0.2, size=x.shape), 0, 1)
    s, v, _ = oracle.ssim(x, y, wh)
    h = 1e-6
    flat = x.reshape(-1)
    for i in range(flat.size):
        old = flat[i]
        flat[i] = old + h
        sp = oracle.ssim(x, y, wh, grad=False)[0]
        flat[i] = old - h
        sm = oracle.ssim(x, y, wh, grad=False)[0]
        flat[i] = old
        assert abs((sp - sm) / (2 * h) - v.reshape(-1)[i]) <= 1e-7 * np.abs(v).max(), i


# ----------------------------------------------------------------- initialisation from SfM points

def test_knn_mean_distance_against_scipy_kdtree():
    from scipy.spatial import cKDTree
    rng = np.random.default_rng(8)
    pts = np.concatenate([rng.normal(0, 0.3, (700, 3)), rng.uniform(-2, 2, (300, 3))])
    d, _ = cKDTree(pts).query(pts, k=5)
    np.testing.assert_allclose(oracle.knn_mean_dist(pts, 4), d[:, 1:].mean(axis=1), rtol=1e-12)
    np.testing.assert_allclose(oracle.knn_mean_dist(pts, 1), d[:, 1], rtol=1e-12)


def test_knn_mean_distance_lattice_and_line_closed_forms():
    a = 0.37
    g = np.arange(5) * a
    lat = np.stack(np.meshgrid(g, g, g, indexing="ij"), -1).reshape(-1, 3)
    d = oracle.knn_mean_dist(lat, 4).reshape(5, 5, 5)
    assert abs(d[2, 2, 2] - a) < 1e-14                       # six neighbours at a
    assert abs(d[0, 0, 0] - (3 + np.sqrt(2)) * a / 4) < 1e-14  # corner: a, a, a, sqrt(2) a
    line = np.zeros((9, 3))
    line[:, 1] = np.arange(9) * a
    d = oracle.knn_mean_dist(line, 4)
    assert abs(d[4] - 1.5 * a) < 1e-14 and abs(d[0] - 2.5 * a) < 1e-14
    # fewer other points than k: all of them
    tri = np.array([[0, 0, 0], [1.0, 0, 0], [0, 2.0, 0]])
    np.testing.assert_allclose(oracle.knn_mean_dist(tri, 4), [1.5, (1 + np.sqrt(5)) / 2, (2 + np.sqrt(5)) / 2],
                               rtol=1e-14)


def test_init_gaussians_closed_forms():
    rng = np.random.default_rng(9)
    pts = rng.uniform(-1, 1, (50, 3))
    pts[7] = pts[3]                                   # coincident pair
    pts[8] = pts[3]
    pts[9] = pts[3]
    pts[10] = pts[3]                                  # five coincident points: distance 0
    rgb = rng.uniform(size=(50, 3))
    g = oracle.init_gaussians(pts, rgb, sh_degree=2, s_min=1e-7)
    np.testing.assert_array_equal(g["means"], pts.T)
    C0 = 1 / (2 * np.sqrt(np.pi))
    np.testing.assert_allclose(0.5 + C0 * g["sh"][0], rgb.T, rtol=1e-14)
    assert np.all(g["sh"][1:] == 0) and g["sh"].shape == (9, 3, 50)
    np.testing.assert_allclose(1 / (1 + np.exp(-g["opacity_logit"])), 0.1, rtol=1e-14)
    np.testing.assert_array_equal(g["quats"][0], 1.0)
    np.testing.assert_array_equal(g["quats"][1:], 0.0)
    d = oracle.knn_mean_dist(pts, 4)
    np.testing.assert_allclose(np.exp(g["log_scales"]), np.broadcast_to(np.maximum(d, 1e-7), (3, 50)),
                               rtol=1e-14)
    assert d[3] == 0.0 and abs(np.exp(g["log_scales"][0, 3]) - 1e-7) < 1e-20


# ----------------------------------------------------------------- bundle adjustment, one LM step

def _ba_problem(seed=50, ncam=4, Pt=30, noise=0.0, perturb=0.0):
    rng = np.random.default_rng(seed)
    vms, intr = [], []
    for i in range(ncam):
        R = Rotation.from_rotvec(rng.normal(0, 0.2, 3)).as_matrix()
        vms.append(_viewmat(R, np.array([0.3 * i, -0.1 * i, 0.0]) + rng.normal(0, 0.05, 3)))
        intr.append([300.0, 310.0, 160.0, 120.0])
    vms, intr = np.array(vms), np.array(intr)
    X = rng.uniform(-1, 1, (Pt, 3)) + np.array([0, 0, 5.0])
    cam, pt, xy = [], [], []
    for k in range(Pt):
        for i in sorted(rng.choice(ncam, size=min(ncam, 3), replace=False)):
            M3 = vms[i].reshape(3, 4)
            p = M3[:, :3] @ X[k] + M3[:, 3]
            cam.append(i)
            pt.append(k)
            xy.append([intr[i, 0] * p[0] / p[2] + intr[i, 2], intr[i, 1] * p[1] / p[2] + intr[i, 3]])
    order = np.argsort(cam, kind="stable")
    cam, pt, xy = np.array(cam)[order], np.array(pt)[order], np.array(xy)[order]
    xy = xy + rng.normal(0, noise, xy.shape) if noise else xy
    if perturb:
        vms = np.stack([_left_perturb(v, rng.normal(0, perturb, 6) * np.array([1, 1, 1, .3, .3, .3]))
                        for v in vms])
        X = X + rng.normal(0, perturb, X.shape)
    return X, vms, intr, cam.astype(np.int32), pt.astype(np.int32), xy


def test_ba_gradient_is_the_track_gradient():
    X, vm, intr, cam, pt, xy = _ba_problem(noise=2.0)       # inliers and outliers
    H, g, cost, masked = oracle.ba_normal(X, vm, intr, cam, pt, xy, delta=1.0)
    t = oracle.track(X, vm, intr, cam, pt, xy, delta=1.0, lam=1.0)
    nc = vm.shape[0]
    np.testing.assert_allclose(g[:6 * nc], t["v_twist"].reshape(-1) / 2, rtol=1e-10, atol=1e-12)
    np.testing.assert_allclose(g[6 * nc:], t["v_X"].reshape(-1) / 2, rtol=1e-10, atol=1e-12)
    assert abs(cost - t["loss"]) <= 1e-10 * cost and masked == 0
    np.testing.assert_allclose(H, H.T, atol=1e-9 * np.abs(H).max())


def test_ba_gauss_newton_matrix_is_the_hessian_at_zero_residual():
    # all observations exact (r = 0, every one an inlier): the Hessian of
    # cost / 2 = sum |r|^2 / 2 is J^T J = H; central differences of g
    X, vm, intr, cam, pt, xy = _ba_problem(seed=51, ncam=3, Pt=8)
    H, g, _, _ = oracle.ba_normal(X, vm, intr, cam, pt, xy)
    assert np.max(np.abs(g)) < 1e-9
    nc = vm.shape[0]
    h = 1e-6
    for col in range(H.shape[0]):
        if col < 6 * nc:
            i, e = divmod(col, 6)
            xi = np.zeros(6)
            xi[e] = h
            vp, vmn = vm.copy(), vm.copy()
            vp[i] = _left_perturb(vm[i], xi)
            vmn[i] = _left_perturb(vm[i], -xi)
            gp = oracle.ba_normal(X, vp, intr, cam, pt, xy)[1]
            gm = oracle.ba_normal(X, vmn, intr, cam, pt, xy)[1]
        else:
            k, e = divmod(col - 6 * nc, 3)
            Xp, Xm = X.copy(), X.copy()
            Xp[k, e] += h
            Xm[k, e] -= h
            gp = oracle.ba_normal(Xp, vm, intr, cam, pt, xy)[1]
            gm = oracle.ba_normal(Xm, vm, intr, cam, pt, xy)[1]
        fd = (gp - gm) / (2 * h)
        assert np.max(np.abs(fd - H[:, col])) <= 1e-6 * np.abs(H).max(), col


def test_ba_lm_steps_converge_and_steepest_descent_limit():
    X, vm, intr, cam, pt, xy = _ba_problem(seed=52, ncam=4, Pt=25, perturb=0.01)
    costs = []
    for it in range(6):
        dtw, dX, cost = oracle.ba_step(X, vm, intr, cam, pt, xy, lm_lambda=1e-6)
        costs.append(cost)
        vm = np.stack([_left_perturb(vm[i], dtw[i]) for i in range(vm.shape[0])])
        X = X + dX
    assert costs[0] > 1.0 and costs[-1] < 1e-12 * costs[0], costs
    assert all(b <= a for a, b in zip(costs, costs[1:]))
    # a large damping turns the step into scaled steepest descent
    X, vm, intr, cam, pt, xy = _ba_problem(seed=53, noise=1.5)
    H, g, _, _ = oracle.ba_normal(X, vm, intr, cam, pt, xy)
    lam = 1e8
    dtw, dX, _ = oracle.ba_step(X, vm, intr, cam, pt, xy, lm_lambda=lam)
    d = np.concatenate([dtw.reshape(-1), dX.reshape(-1)])
    np.testing.assert_allclose(d * lam * np.diag(H), -g, rtol=1e-6, atol=1e-9 * np.abs(g).max())


def test_ba_normal_residual_matches_the_dense_system():
    X, vm, intr, cam, pt, xy = _ba_problem(seed=54, noise=1.5)
    H, g, _, _ = oracle.ba_normal(X, vm, intr, cam, pt, xy)
    rng = np.random.default_rng(0)
    nc = vm.shape[0]
    d = rng.normal(size=g.shape)
    rc, rp = oracle.ba_normal_residual(X, vm, intr, cam, pt, xy, d[:6 * nc], d[6 * nc:], lm_lambda=0.3)
    want = (H + 0.3 * np.diag(np.diag(H))) @ d + g
    np.testing.assert_allclose(np.concatenate([rc.reshape(-1), rp.reshape(-1)]), want, rtol=1e-10,
                               atol=1e-10 * np.abs(want).max())
    dtw, dX, _ = oracle.ba_step(X, vm, intr, cam, pt, xy, lm_lambda=0.3)
    rc, rp = oracle.ba_normal_residual(X, vm, intr, cam, pt, xy, dtw, dX, lm_lambda=0.3)
    assert np.max(np.abs(np.concatenate([rc.reshape(-1), rp.reshape(-1)]))) <= 1e-9 * np.abs(g).max()


# ----------------------------------------------------------------- MCMC relocation and noise

def _mcmc_scene(N, rng, sh_degree=1, logit=None):
    K = (sh_degree + 1) ** 2
    g = dict(means=rng.normal(size=(3, N)), log_scales=rng.normal(-3, 0.3, (3, N)),
             quats=rng.normal(size=(4, N)), opacity_logit=rng.normal(0, 2, N) if logit is None else logit,
             sh=rng.normal(0, 0.2, (K, 3, N)))
    m1 = {k: rng.normal(size=v.shape) for k, v in g.items()}
    m2 = {k: rng.uniform(size=v.shape) for k, v in g.items()}
    return g, (m1, m2)


@pytest.mark.parametrize("o", [0.05, 0.3, 0.9])
@pytest.mark.parametrize("n", [1, 2, 3, 6])
def test_mcmc_copies_keep_centre_opacity_and_axis_integral(o, n):
    # one live Gaussian (opacity o) and n - 1 dead ones: all move onto it, so
    # n copies share it; their combined opacity at the centre is o, and the
    # integral of the combined opacity along an axis equals o sigma sqrt(2 pi)
    from scipy.integrate import quad
    rng = np.random.default_rng(n)
    logit = np.concatenate([[np.log(o / (1 - o))], np.full(n - 1, -8.0)])
    g, mom = _mcmc_scene(n, rng, logit=logit)
    u = rng.uniform(size=n)
    G, M, src, moved = oracle.mcmc_relocate(g, mom, u, 1)
    assert moved == n - 1 and np.all(src[1:] == 0) and src[0] == -1
    op = 1 / (1 + np.exp(-G["opacity_logit"]))
    np.testing.assert_allclose(op, op[0], rtol=1e-12)
    assert abs(1 - (1 - op[0]) ** n - o) < 1e-12
    f = np.exp(G["log_scales"][0, 0] - g["log_scales"][0, 0])
    sig = 0.7
    integ, _ = quad(lambda x: 1 - (1 - op[0] * np.exp(-x * x / (2 * (sig * f) ** 2))) ** n, -np.inf, np.inf,
                    epsabs=1e-13, epsrel=1e-12)
    assert abs(integ - o * sig * np.sqrt(2 * np.pi)) <= 1e-9
    # copies carry the source; every touched moment restarts at zero
    for k in ("means", "quats", "sh", "log_scales"):
        assert np.all(G[k][..., 1:] == G[k][..., :1]), k
    np.testing.assert_array_equal(G["means"][:, 0], g["means"][:, 0])
    if n > 1:
        for k in M[0]:
            assert np.all(M[0][k] == 0) and np.all(M[1][k] == 0), k


def test_mcmc_draws_follow_the_integer_opacity_weights():
    rng = np.random.default_rng(60)
    N = 4000
    g, mom = _mcmc_scene(N, rng)
    o = 1 / (1 + np.exp(-g["opacity_logit"]))
    dead = o <= 0.005
    g["opacity_logit"][rng.choice(N, 1500, replace=False)] = -9.0    # many dead ones
    o = 1 / (1 + np.exp(-g["opacity_logit"]))
    dead = o <= 0.005
    u = rng.uniform(size=N)
    G, M, src, moved = oracle.mcmc_relocate(g, mom, u, 1)
    assert moved == dead.sum()
    # independent draw: numpy cumulative sum of the integer weights
    w = np.where(dead, 0, np.floor(o * 2 ** 24)).astype(np.int64)
    cdf = np.cumsum(w)
    want = np.searchsorted(cdf, np.floor(u * float(cdf[-1])).astype(np.int64), side="right")
    np.testing.assert_array_equal(src[dead], want[dead])
    assert np.all(src[~dead] == -1)
    # never a dead source; the untouched live Gaussians keep everything
    assert not np.any(dead[src[dead]])
    untouched = ~dead & ~np.isin(np.arange(N), src[dead])
    for k in g:
        np.testing.assert_array_equal(G[k][..., untouched], g[k][..., untouched])
        np.testing.assert_array_equal(M[0][k][..., untouched], mom[0][k][..., untouched])


def test_mcmc_draw_frequencies_match_opacity():
    # 200k draws onto 5 live Gaussians: frequencies within 5 sigma of o / sum o
    # (each source far past the cap of 51 copies in the opacity rule)
    rng = np.random.default_rng(61)
    logit = np.concatenate([[-2.0, -0.5, 0.0, 1.0, 3.0], np.full(200_000, -9.0)])
    g, mom = _mcmc_scene(logit.size, rng, sh_degree=0, logit=logit)
    G, M, src, moved = oracle.mcmc_relocate(g, mom, rng.uniform(size=logit.size), 0)
    o = 1 / (1 + np.exp(-logit[:5]))
    p = o / o.sum()
    cnt = np.bincount(src[5:], minlength=5)
    assert np.all(np.abs(cnt - 200_000 * p) <= 5 * np.sqrt(200_000 * p * (1 - p)))


def test_mcmc_nothing_to_move():
    rng = np.random.default_rng(62)
    g, mom = _mcmc_scene(50, rng, logit=np.full(50, 1.0))          # all alive
    G, M, src, moved = oracle.mcmc_relocate(g, mom, rng.uniform(size=50), 1)
    assert moved == 0 and np.all(src == -1)
    g, mom = _mcmc_scene(50, rng, logit=np.full(50, -9.0))         # all dead
    G, M, src, moved = oracle.mcmc_relocate(g, mom, rng.uniform(size=50), 1)
    assert moved == 0
    for k in g:
        np.testing.assert_array_equal(G[k], g[k])


def test_mcmc_noise_closed_form():
    rng = np.random.default_rng(63)
    N = 40
    # opacities around the dead threshold, where the gate is neither 0 nor 1
    o0 = rng.uniform(0.001, 0.03, N)
    g, _ = _mcmc_scene(N, rng, logit=np.log(o0 / (1 - o0)))
    g["quats"] = np.tile([[2.0], [0.0], [0.0], [0.0]], (1, N))        # identity rotation
    s = np.exp(rng.normal(-2, 0.2, N))
    g["log_scales"] = np.tile(np.log(s), (3, 1))
    eta = rng.normal(size=(3, N))
    out = oracle.mcmc_noise(g, eta, scale=3.0, k=100.0, t=0.005)
    o = 1 / (1 + np.exp(-g["opacity_logit"]))
    gate = 1 / (1 + np.exp(100 * (o - 0.005)))
    np.testing.assert_allclose(out - g["means"], 3.0 * gate * s ** 2 * eta, rtol=1e-9, atol=1e-15)
    # a rotated anisotropic Gaussian: the displacement is Sigma eta
    g2 = dict(g)
    R = Rotation.random(random_state=3)
    qx, qy, qz, qw = R.as_quat()
    g2["quats"] = np.tile([[qw], [qx], [qy], [qz]], (1, N))
    ls = np.log(np.array([0.1, 0.02, 0.3]))
    g2["log_scales"] = np.tile(ls[:, None], (1, N))
    out = oracle.mcmc_noise(g2, eta, scale=1.0)
    Sig = R.as_matrix() @ np.diag(np.exp(2 * ls)) @ R.as_matrix().T
    np.testing.assert_allclose(out - g2["means"], (Sig @ eta) * gate, rtol=1e-10, atol=1e-15)


def test_mcmc_copy_count_cap():
    # 60 dead Gaussians onto one live one: 61 copies, the opacity rule at n = 51
    rng = np.random.default_rng(64)
    o = 0.6
    g, mom = _mcmc_scene(61, rng, logit=np.concatenate([[np.log(o / (1 - o))], np.full(60, -9.0)]))
    G, M, src, moved = oracle.mcmc_relocate(g, mom, rng.uniform(size=61), 1)
    assert moved == 60
    op = 1 / (1 + np.exp(-G["opacity_logit"]))
    np.testing.assert_allclose(op, 1 - (1 - o) ** (1 / 51), rtol=1e-12)
