"""Pins of the oracle ray marcher against closed forms, invariants and brute force.

The paper gives the renderer only as a ray marcher (Methods, "Foveated
Rendering"); the per-ray rules are the readings documented in the ABI header:
midpoint segments with a partial last one, clamp-to-edge trilinear, linear TF
lookup of (rgb, extinction), central-difference Blinn-Phong, front-to-back
compositing with early termination.
"""
import math

import numpy as np
import pytest

import oracle
import synthetic
from tests import brute


def f32(x):
    return float(np.float32(x))


def const_tf(rgb, sigma):
    tf = np.zeros((256, 4), np.float32)
    tf[:, :3] = rgb
    tf[:, 3] = sigma
    return tf


AXIAL = dict(eye=(0.0, 0.0, 2.0), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fovy_deg=45.0,
             eye_offset=0.0)


def test_empty_volume_returns_background_exactly():
    vol = np.zeros((12, 10, 9), np.uint8)
    tf = synthetic.tf_blob(1)
    assert tf[0, 3] == 0.0
    mp = synthetic.march_params(shading=True, bg=(0.1, 0.2, 0.3))
    cams = [synthetic.orbit_camera(k) for k in (0, 7)]
    out = oracle.march(vol, tf, cams, 24, 16, mp)
    bg = np.array([f32(0.1), f32(0.2), f32(0.3)])
    assert np.all(out["rgba"][:, :3] == bg)
    assert np.all(out["rgba"][:, 3] == 0.0)
    assert np.all(out["depth"] == 0.0)


@pytest.mark.parametrize("shading", [0, 1])
def test_homogeneous_axial_transmittance(shading):
    """Constant volume + constant TF: A = 1 - exp(-sigma L) with L = n_z voxels along the
    axis; RGB = c A + bg (1 - A) (ka c with shading: zero gradient)."""
    n = 16
    vol = np.full((n, n, n), 0.5, np.float32)
    rgb, sigma = (0.3, 0.6, 0.9), 0.05
    tf = const_tf(rgb, sigma)
    mp = synthetic.march_params(shading=shading, alpha_stop=1.0, bg=(0.25, 0.5, 0.75))
    out = oracle.march(vol, tf, [AXIAL], 3, 3, mp, idx=np.array([4], np.uint32))
    A = 1 - math.exp(-f32(sigma) * n)
    c = np.array([f32(v) for v in rgb]) * (f32(0.2) if shading else 1.0)
    bg = np.array([f32(0.25), f32(0.5), f32(0.75)])
    np.testing.assert_allclose(out["rgba"][0, 3], A, rtol=0, atol=1e-12)
    np.testing.assert_allclose(out["rgba"][0, :3], c * A + bg * (1 - A), rtol=0, atol=1e-12)
    assert out["samples"][0] == math.ceil(n / 0.5)


def test_homogeneous_oblique_rays_partial_segments():
    """For any ray, A = 1 - exp(-sigma L) exactly thanks to the partial last segment; L from
    an independent face-by-face box intersection; sample count = ceil(L / step)."""
    vol = np.full((7, 11, 13), 200, np.uint8)
    tf = const_tf((0.5, 0.5, 0.5), 0.03)
    mp = synthetic.march_params(alpha_stop=1.0, step_vox=0.37)
    cam = synthetic.orbit_camera(5, phi_deg=31.0)
    W, H = 20, 14
    out = oracle.march(vol, tf, [cam], W, H, mp)
    hits = 0
    for i in range(W * H):
        y, x = divmod(i, W)
        o, d = brute.camera_ray(cam, W, H, x, y)
        iv = brute.box_interval((13, 11, 7), o, d)
        if iv is None:
            assert out["rgba"][i, 3] == 0.0
            continue
        hits += 1
        L = (iv[1] - iv[0]) * 13
        assert abs(out["rgba"][i, 3] - (1 - math.exp(-f32(0.03) * L))) < 1e-9
        assert out["samples"][i] == math.ceil(L / f32(0.37) - 1e-9)
    assert hits > 20


def test_early_termination_closed_form():
    """sigma l = 0.25 per segment: stop at the first k with 1 - exp(-0.25 k) >= 0.99,
    k* = ceil(ln(100) / 0.25) = 19 samples."""
    n = 16
    vol = np.full((n, n, n), 1.0, np.float32)
    tf = const_tf((1.0, 0.5, 0.25), 0.5)
    mp = synthetic.march_params(alpha_stop=0.99)
    out = oracle.march(vol, tf, [AXIAL], 3, 3, mp, idx=np.array([4], np.uint32))
    assert out["samples"][0] == 19
    A = 1 - math.exp(-0.25 * 19)
    assert abs(out["rgba"][0, 3] - A) < 1e-12
    np.testing.assert_allclose(out["rgba"][0, :3], np.array([1.0, 0.5, 0.25]) * A, atol=1e-12)


def test_linear_ramp_shading_closed_form():
    """v = a x + b along x, ray along -z through the centre: the trilinear field is exact
    and the central difference is (a, 0, 0) everywhere on the ray, so every sample has the
    same Blinn-Phong colour c (ka + kd |n.L|) + ks |n.H|^32 with n = -x^."""
    n = 16
    x = np.arange(n, dtype=np.float64)
    vol = np.broadcast_to((0.02 * x + 0.1).astype(np.float32), (n, n, n)).copy()
    rgb, sigma = np.array([0.8, 0.4, 0.2]), 0.04
    tf = const_tf(rgb, sigma)
    mp = synthetic.march_params(shading=True, alpha_stop=1.0)
    out = oracle.march(vol, tf, [AXIAL], 3, 3, mp, idx=np.array([4], np.uint32))
    Lh = np.ones(3) / math.sqrt(3)
    Hv = Lh + np.array([0, 0, 1.0])
    Hv /= np.linalg.norm(Hv)
    nrm = np.array([-1.0, 0, 0])
    c = rgb.astype(np.float32) * (f32(0.2) + f32(0.7) * abs(nrm @ Lh)) + \
        f32(0.3) * abs(nrm @ Hv) ** 32
    A = 1 - math.exp(-f32(sigma) * n)
    np.testing.assert_allclose(out["rgba"][0, :3], c * A, atol=1e-12)


def test_trilinear_exact_on_linear_field_and_clamp():
    n = 9
    zz, yy, xx = np.mgrid[0:n, 0:n, 0:n].astype(np.float64)
    vol = (0.01 * xx + 0.02 * yy + 0.03 * zz + 0.05).astype(np.float32)
    rng = np.random.default_rng(0)
    for _ in range(50):
        q = rng.uniform(0, n - 1, 3)
        want = 0.01 * q[0] + 0.02 * q[1] + 0.03 * q[2] + 0.05
        assert abs(oracle.sample(vol, q) - want) < 1e-6  # float32 voxel rounding
    # voxel centres exactly; clamp-to-edge outside
    assert oracle.sample(vol, (3, 4, 5)) == float(vol[5, 4, 3])
    assert oracle.sample(vol, (-0.7, 4, 5)) == float(vol[5, 4, 0])
    assert oracle.sample(vol, (n - 1 + 0.4, 0, n + 3)) == float(vol[n - 1, 0, n - 1])


def test_half_float_decoding():
    vals = np.array([0.0, 1e-7, 6.1e-5, 0.333, 0.5, 0.999, 1.0, 65504.0, -2.5], np.float16)
    vol = vals.reshape(1, 1, -1)
    for i, v in enumerate(vals):
        assert oracle.sample(vol, (i, 0, 0)) == float(v)


def test_opacity_monotone_in_alpha_stop():
    vol = synthetic.blob_volume(1001, 24)
    tf = synthetic.tf_blob(1001)
    cam = synthetic.orbit_camera(11)
    prev = None
    for stop in (0.3, 0.6, 0.9, 0.99, 1.0):
        out = oracle.march(vol, tf, [cam], 16, 16, synthetic.march_params(alpha_stop=stop))
        if prev is not None:
            assert np.all(out["rgba"][:, 3] >= prev - 1e-15)
        prev = out["rgba"][:, 3]


def test_mirror_symmetry():
    """Volume mirrored in x, camera and light in the x = 0 plane: the image is mirrored."""
    vol = synthetic.value_noise_volume(7, n=16, octaves=3, base_period=8)
    tf = synthetic.tf_noise(7)
    cam = dict(eye=(0.0, 0.6, 1.9), target=(0.0, 0.0, 0.0), up=(0.0, 1.0, 0.0), fovy_deg=45.0,
               eye_offset=0.0)
    mp = synthetic.march_params(shading=True, light_dir=(0.0, 1.0, 0.5))
    W, H = 18, 12
    a = oracle.march(vol, tf, [cam], W, H, mp)["rgba"].reshape(H, W, 4)
    b = oracle.march(vol[:, :, ::-1].copy(), tf, [cam], W, H, mp)["rgba"].reshape(H, W, 4)
    np.testing.assert_allclose(a, b[:, ::-1], atol=1e-12)


@pytest.mark.parametrize("shading,dtype", [(0, np.uint8), (1, np.float32)])
def test_bruteforce_8cube(shading, dtype):
    """Literal O(N^2) re-derivation on 8^3 volumes agrees with the oracle to 1e-12."""
    rng = np.random.default_rng(3 + shading)
    if dtype == np.uint8:
        vol = rng.integers(0, 256, (8, 8, 8)).astype(np.uint8)
        tf = synthetic.tf_blob(5)
        tf[:, 3] *= 6  # make the tiny volume visibly opaque
    else:
        vol = rng.uniform(0, 1, (8, 8, 8)).astype(np.float32)
        tf = synthetic.tf_noise(5)
        tf[:, 3] *= 8
    cam = synthetic.orbit_camera(rng.integers(60), phi_deg=float(rng.uniform(-50, 50)))
    mp = synthetic.march_params(shading=shading, alpha_stop=0.9, bg=(0.1, 0.0, 0.2))
    W, H = 12, 10
    out = oracle.march(vol, tf, [cam], W, H, mp)
    for i in range(W * H):
        y, x = divmod(i, W)
        r = brute.pixel(vol, tf, cam, W, H, x, y, mp)
        np.testing.assert_allclose(out["rgba"][i], r[:4], atol=1e-12, rtol=0)
        assert out["samples"][i] == r[4]


def test_stereo_offset_shifts_origin():
    """eye_offset moves the origin along the camera's right axis; view 1 is independent."""
    vol = synthetic.blob_volume(1002, 16)
    tf = synthetic.tf_blob(1002)
    c0 = synthetic.orbit_camera(0, eye_offset=-0.032)
    c1 = synthetic.orbit_camera(0, eye_offset=0.032)
    mp = synthetic.march_params()
    both = oracle.march(vol, tf, [c0, c1], 10, 8, mp)["rgba"]
    a = oracle.march(vol, tf, [c0], 10, 8, mp)["rgba"]
    b = oracle.march(vol, tf, [c1], 10, 8, mp)["rgba"]
    np.testing.assert_array_equal(both[:80], a)
    np.testing.assert_array_equal(both[80:], b)
    for i in range(80):
        y, x = divmod(i, 10)
        r = brute.pixel(vol, tf, c1, 10, 8, x, y, mp)
        np.testing.assert_allclose(b[i], r[:4], atol=1e-12)


def test_ambiguity_flags_mark_threshold_rays():
    """Rays whose stopping decision lies within eps of alpha_stop are flagged and both
    branches are returned."""
    vol = synthetic.blob_volume(1003, 24)
    tf = synthetic.tf_blob(1003)
    cam = synthetic.orbit_camera(3)
    mp = synthetic.march_params(alpha_stop=0.5)
    out = oracle.march(vol, tf, [cam], 32, 32, mp, alts=True, eps=0.02)
    f = out["flags"].astype(bool)
    assert f.any()
    assert np.all(out["rgba_lo"][f, 3] <= out["rgba_hi"][f, 3])
    assert np.array_equal(out["rgba_lo"][~f], out["rgba_hi"][~f])


# ------------------------------------------------------------------ shadows
# Global ray-marched shadows (Methods, "Foveated Rendering": one shadow ray
# per sample towards the light, at a quarter of the primary sample rate).
# Reading: directional light; the shadow ray runs from the sample to where it
# leaves the box, midpoint segments of shadow_step voxel lengths (the last
# shorter), transmittance exp(-sum sigma_j len_j) scaling the diffuse and
# specular terms.

@pytest.mark.parametrize("ds", [0.5, 2.0, 3.7])
def test_shadow_constant_extinction_closed_form(ds):
    """With the same extinction c everywhere, the transmittance is exp(-c L)
    for the exit distance L of the box [-1/2, n - 1/2]^3, whatever the
    segment length."""
    vol = np.full((12, 10, 8), 0.3, np.float32)  # nz, ny, nx
    c = 0.07
    tf = const_tf((1, 1, 1), c)
    c = f32(c)
    # along +x from x = 3: the face x = 7.5 is 4.5 away
    t = oracle.shadow_at(vol, tf, (3.0, 2.0, 5.0), (1, 0, 0), ds)
    assert t == pytest.approx(math.exp(-c * 4.5), rel=1e-13)
    # along -y from y = 2.25: the face y = -0.5 is 2.75 away
    t = oracle.shadow_at(vol, tf, (3.0, 2.25, 5.0), (0, -1, 0), ds)
    assert t == pytest.approx(math.exp(-c * 2.75), rel=1e-13)
    # diagonal from (1, 2, 3): faces 7.5, 9.5, 11.5 -> min(6.5, 7.5, 8.5) sqrt(3)
    t = oracle.shadow_at(vol, tf, (1.0, 2.0, 3.0), (1, 1, 1), ds)
    assert t == pytest.approx(math.exp(-c * 6.5 * math.sqrt(3)), rel=1e-12)


@pytest.mark.parametrize("direction", [1, -1])
def test_shadow_slab_integral_exact(direction):
    """A one-voxel-thick wall (value 1 on the planes x = 4 and 5, 0 elsewhere)
    seen through a linear TF sigma = c v: the trilinear field along x is a
    trapezoid with integral 2, and half-voxel midpoint segments that start on
    a voxel plane integrate it exactly, so T = exp(-2 c) from either side."""
    vol = np.zeros((4, 4, 10), np.float32)
    vol[:, :, 4:6] = 1.0
    c = 0.3
    tf = np.zeros((256, 4), np.float32)
    tf[:, 3] = c * np.arange(256) / 255.0
    x0 = 1.0 if direction > 0 else 8.0
    t = oracle.shadow_at(vol, tf, (x0, 1.5, 2.0), (direction, 0, 0), 0.5)
    sig = tf[:, 3].astype(np.float64)
    # the TF's float32 entries are linear in the index up to rounding
    assert t == pytest.approx(math.exp(-2 * c), rel=1e-6)
    # beyond the wall, looking away from it: nothing in the way
    xb = 7.0 if direction > 0 else 2.0
    assert oracle.shadow_at(vol, tf, (xb, 1.5, 2.0), (direction, 0, 0), 0.5) == 1.0
    assert sig[0] == 0.0


def test_shadow_marching_closed_form():
    """The linear ramp v = a x + b (constant colour and extinction c) seen along -z with
    the light along (1, 1, 1): every sample has the same normal -x^, and its shadow ray
    leaves the box through the face it meets first, so each sample's light is scaled by
    exp(-c L_k) with L_k from the geometry alone."""
    n = 16
    x = np.arange(n, dtype=np.float64)
    vol = np.broadcast_to((0.02 * x + 0.1).astype(np.float32), (n, n, n)).copy()
    rgb, sigma = np.array([0.8, 0.4, 0.2]), 0.04
    tf = const_tf(rgb, sigma)
    mp = synthetic.march_params(shading=True, alpha_stop=1.0, shadow_step=2.0)
    W = H = 3
    out = oracle.march(vol, tf, [AXIAL], W, H, mp, idx=np.array([4], np.uint32))
    c = f32(sigma)
    Lh = np.ones(3) / math.sqrt(3)
    Hv = Lh + np.array([0, 0, 1.0])
    Hv /= np.linalg.norm(Hv)
    nrm = np.array([-1.0, 0, 0])
    # the centre pixel's ray: x = y = 7.5 (index space), z from n - 1/2 down to -1/2;
    # sample k sits at z = n - 1/2 - (k + 1/2) * 0.5 (16 voxels / 0.5 = 32 segments)
    total = np.zeros(3)
    T = 1.0
    a = 1 - math.exp(-c * 0.5)
    for k in range(32):
        z = n - 0.5 - (k + 0.5) * 0.5
        L = min(n - 0.5 - 7.5, n - 0.5 - 7.5, n - 0.5 - z) * math.sqrt(3)
        ts = math.exp(-c * L)
        col = rgb.astype(np.float32) * (f32(0.2) + ts * f32(0.7) * abs(nrm @ Lh)) + \
            ts * f32(0.3) * abs(nrm @ Hv) ** 32
        total += T * a * col
        T *= 1 - a
    np.testing.assert_allclose(out["rgba"][0, :3], total, atol=1e-12)


def test_shadows_only_darken():
    """Shadows scale the diffuse and specular light by a transmittance in [0, 1]: on a
    black background every colour channel can only drop, and opacity, depth and the
    sample count do not change.  shadow_step = 0 is the unshadowed march, bit for bit."""
    vol = synthetic.value_noise_volume(17, n=24, octaves=3, base_period=8)
    tf = synthetic.tf_noise(17)
    tf[:, 3] *= 4
    cam = synthetic.orbit_camera(11)
    W, H = 20, 14
    plain = oracle.march(vol, tf, [cam], W, H, synthetic.march_params(shading=True))
    zero = oracle.march(vol, tf, [cam], W, H,
                        synthetic.march_params(shading=True, shadow_step=0.0))
    shad = oracle.march(vol, tf, [cam], W, H,
                        synthetic.march_params(shading=True, shadow_step=2.0))
    assert np.array_equal(plain["rgba"], zero["rgba"])
    assert np.all(shad["rgba"][:, :3] <= plain["rgba"][:, :3] + 1e-15)
    assert (shad["rgba"][:, :3] < plain["rgba"][:, :3] - 1e-6).any()
    np.testing.assert_array_equal(shad["rgba"][:, 3], plain["rgba"][:, 3])
    np.testing.assert_array_equal(shad["depth"], plain["depth"])
    np.testing.assert_array_equal(shad["samples"], plain["samples"])


# ------------------------------------------------------------------ depth
# The premultiplied depth D = sum_k T_k alpha_k t_k, with t_k the distance of
# sample k from the ray's origin (world units), is pinned on the centre pixel
# of the axial camera: the ray runs along -z from z = 2, enters the unit box
# at t0 = 1.5 and every sample sits at t_k = t0 + h m_k (h = 1/n, m_k the
# segment's midpoint in voxel lengths).  With a constant extinction sigma the
# sums are geometric series, evaluated here in closed form.

def _axial_depth_closed_form(n, sigma, step, K=None):
    """D for the constant medium: full segments k < N - 1 of length `step`, the
    last one of length L - (N - 1) step, the ray stopped after K samples."""
    L = float(n)
    N = math.ceil(L / step - 1e-12)
    K = N if K is None else K
    h, t0 = 1.0 / n, 1.5
    r = math.exp(-sigma * step)
    a = 1.0 - r
    kf = min(K, N - 1)  # full segments composited
    s0 = (1 - r ** kf) / (1 - r)
    s1 = r * (1 - kf * r ** (kf - 1) + (kf - 1) * r ** kf) / (1 - r) ** 2
    D = a * ((t0 + h * step / 2) * s0 + h * step * s1)
    if K == N:  # the partial last segment
        ll = L - (N - 1) * step
        D += r ** (N - 1) * (1 - math.exp(-sigma * ll)) * (t0 + h * ((N - 1) * step + ll / 2))
    return D


@pytest.mark.parametrize("step", [0.5, 0.37])
def test_depth_homogeneous_axial_closed_form(step):
    """No early termination: every segment composited, the partial last one
    (step 0.37: 43 full segments and one of 0.09 voxels) included."""
    n = 16
    vol = np.full((n, n, n), 0.5, np.float32)
    tf = const_tf((0.3, 0.6, 0.9), 0.05)
    mp = synthetic.march_params(alpha_stop=1.0, step_vox=step)
    out = oracle.march(vol, tf, [AXIAL], 3, 3, mp, idx=np.array([4], np.uint32))
    want = _axial_depth_closed_form(n, f32(0.05), f32(step))
    assert out["samples"][0] == math.ceil(n / f32(step))
    assert abs(out["depth"][0] - want) < 1e-12
    # the depth is a weighted mean distance times the opacity: between the
    # box entry and exit distances
    A = out["rgba"][0, 3]
    assert 1.5 * A < out["depth"][0] < 2.5 * A


def test_depth_early_termination_closed_form():
    """sigma l = 0.25: the ray stops after 19 samples (see the opacity pin);
    D sums only those."""
    n = 16
    vol = np.full((n, n, n), 1.0, np.float32)
    tf = const_tf((1.0, 0.5, 0.25), 0.5)
    mp = synthetic.march_params(alpha_stop=0.99)
    out = oracle.march(vol, tf, [AXIAL], 3, 3, mp, idx=np.array([4], np.uint32))
    assert out["samples"][0] == 19
    want = _axial_depth_closed_form(n, 0.5, 0.5, K=19)
    assert abs(out["depth"][0] - want) < 1e-12
    # a slip that measured t from the box entry would give D - t0 A
    assert abs(out["depth"][0] - (want - 1.5 * out["rgba"][0, 3])) > 1.0


def test_depth_single_opaque_voxel_plane():
    """One plane of ones (z index 5) in an empty 16^3 volume, a TF with extinction
    2 above v ~ 0.7 and 0 below.  Along the axis the field is the triangle
    1 - |z - 5|, and the samples sit at quarter-voxel offsets from the voxel
    planes, so exactly two of them see v = 0.75: z = 5.25 and then 4.75 (index
    space; the ray runs from z = n - 1/2 down).  Each is at the world distance
    t = 2 - (z - 7.5) h from the eye."""
    n = 16
    vol = np.zeros((n, n, n), np.float32)
    vol[5] = 1.0
    tf = np.zeros((256, 4), np.float32)
    tf[:, :3] = 1.0
    tf[int(0.7 * 255) + 1:, 3] = 2.0  # entries above v ~ 0.7
    mp = synthetic.march_params(alpha_stop=1.0)
    out = oracle.march(vol, tf, [AXIAL], 3, 3, mp, idx=np.array([4], np.uint32))
    h = 1.0 / n
    # the ray meets z index 5.25 first (it runs from z = n - 1/2 downwards)
    a = 1 - math.exp(-f32(2.0) * 0.5)
    t1 = 2.0 - (5.25 - 7.5) * h
    t2 = 2.0 - (4.75 - 7.5) * h
    want = a * t1 + (1 - a) * a * t2
    assert abs(out["depth"][0] - want) < 1e-12
    assert abs(out["rgba"][0, 3] - (1 - (1 - a) ** 2)) < 1e-12


def test_pack_input_literal():
    """Network input per pixel [M r, M g, M b, M, M depth / 2]: two pixels, the
    first sampled, the second not (its colour and depth must not leak)."""
    rgba = np.array([[0.1, 0.2, 0.3, 0.4], [0.5, 0.6, 0.7, 0.8]])
    mask = np.array([1, 0], np.uint8)
    depth = np.array([3.0, 5.0])
    got = oracle.pack_input(rgba, mask, depth)
    want = np.array([[0.1, 0.2, 0.3, 1.0, 1.5], [0.0, 0.0, 0.0, 0.0, 0.0]])
    assert np.array_equal(got, want)
    # any non-zero mask byte counts as sampled
    got = oracle.pack_input(rgba[::-1], np.array([0, 7], np.uint8), depth[::-1])
    assert np.array_equal(got, np.array([[0.0] * 5, [0.1, 0.2, 0.3, 1.0, 1.5]]))
