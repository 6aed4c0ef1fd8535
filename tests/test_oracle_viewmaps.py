"""Pins of the oracle's backprojection precompute (Sec. 7.4, TextureGen Postprocessing): image
coordinates of a plane's texels against the pinhole projection in closed form,
the round trip through the camera ray, the incidence of a plane, back faces,
texels outside the image, and the depth-buffer visibility under an occluder."""
import math

import numpy as np

from planes import textured_plane as plane_mesh

TAN30 = math.tan(math.radians(30.0))


def test_plane_projection_and_incidence_closed_form(oracle_lib):
    V, F, UV = plane_mesh()
    eye = np.array([[0.4, 0.55, 1.5]], np.float32)
    tg = eye[0].astype(np.float64) * [1, 1, 0]
    tan_half, R = math.tan(math.radians(15.0)), 256
    vm = oracle_lib.view_maps(V, F, UV, 64, eye, tg, tan_half, R, 5.0, 1e-3, method="brute")
    p = vm.P
    e = eye[0].astype(np.float64)
    h = e[2]
    col = (-(p[:, 1] - e[1]) / (h * tan_half) + 1) * R / 2 - 0.5
    row = (1 - (p[:, 0] - e[0]) / (h * tan_half)) * R / 2 - 0.5
    inside = (col >= -0.5) & (col < R - 0.5) & (row >= -0.5) & (row < R - 0.5)
    assert 0.2 < inside.mean() < 0.9  # some texels fall outside the narrow view
    assert np.allclose(vm.uv[0, inside], np.stack([col, row], 1)[inside], atol=1e-9)
    assert np.all(vm.uv[0, ~inside] == -1) and np.all(vm.inc[0, ~inside] == 0)
    inc = h / np.linalg.norm(e - p, axis=1)
    assert np.allclose(vm.inc[0, inside], inc[inside], atol=1e-12)


def test_round_trip_through_the_camera_ray(oracle_lib):
    """The camera ray at the (fractional) image coordinates of a texel points
    at the texel: the projection inverts the pixel-ray formula."""
    V, F, UV = plane_mesh()
    V[:, 2] = 0.1 * np.sin(3 * V[:, 0]) * np.cos(2 * V[:, 1])  # not flat
    eyes = np.array([[1.9, -0.4, 1.2], [-0.7, 2.1, 0.9]], np.float32)
    tg = np.array([0.5, 0.5, 0.0])
    vm = oracle_lib.view_maps(V, F, UV, 64, eyes, tg, TAN30, 128, 6.0, 1e-3, method="brute")
    for k in range(2):
        e = eyes[k].astype(np.float64)
        f = tg - e
        f /= np.linalg.norm(f)
        a = np.eye(3)[np.argmin(np.abs(f))]
        r = np.cross(f, a)
        r /= np.linalg.norm(r)
        u = np.cross(r, f)
        ins = vm.uv[k, :, 0] >= -0.5
        col, row = vm.uv[k, ins, 0], vm.uv[k, ins, 1]
        x = ((col + 0.5) * 2 / 128 - 1) * TAN30
        y = (1 - (row + 0.5) * 2 / 128) * TAN30
        d = f + x[:, None] * r + y[:, None] * u
        d /= np.linalg.norm(d, axis=1, keepdims=True)
        q = vm.P[ins] - e
        q /= np.linalg.norm(q, axis=1, keepdims=True)
        assert ins.sum() > 100 and np.abs(d - q).max() < 1e-12


def test_back_faces_have_no_incidence(oracle_lib):
    V, F, UV = plane_mesh()
    eye = np.array([[0.5, 0.5, -1.5]], np.float32)
    vm = oracle_lib.view_maps(V, F, UV, 64, eye, eye[0].astype(np.float64) * [1, 1, 0], TAN30, 128, 5.0, 1e-3,
                              method="brute")
    assert np.all(vm.uv[0, :, 0] >= -0.5)  # every texel projects into the image
    assert np.all(vm.inc == 0)


def test_occluder_zeroes_the_incidence_behind_it(oracle_lib):
    V, F, UV = plane_mesh(occluder=True)
    eye = np.array([[0.45, 0.5, 1.6]], np.float32)
    e = eye[0].astype(np.float64)
    R = 256
    vm = oracle_lib.view_maps(V, F, UV, 128, eye, e * [1, 1, 0], TAN30, R, 5.0, 1e-3, method="brute")
    p = vm.P
    plane = np.abs(p[:, 2]) < 1e-6
    # where the segment from the eye to p meets z = 0.5
    s = (e[2] - 0.5) / (e[2] - p[:, 2])
    hx, hy = e[0] + s * (p[:, 0] - e[0]), e[1] + s * (p[:, 1] - e[1])
    # margin: a few pixels of the depth buffer at the occluder's height
    m = 3 * 2 * 1.1 * TAN30 / R
    inside = (hx > 0.3 + m) & (hx < 0.6 - m) & (hy > 0.2 + m) & (hy < 0.7 - m)
    outside = (hx < 0.3 - m) | (hx > 0.6 + m) | (hy < 0.2 - m) | (hy > 0.7 + m)
    assert (plane & inside).sum() > 200 and (plane & outside).sum() > 1000
    assert np.all(vm.inc[0, plane & inside] == 0)
    assert np.all(vm.inc[0, plane & outside] > 0.5)
    # the occluder itself is seen (it is the nearest surface there)
    top = np.abs(p[:, 2] - 0.5) < 1e-6
    assert top.sum() > 100 and np.all(vm.inc[0, top] > 0.5)
