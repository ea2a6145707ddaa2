"""Pins for the oracle's detector-frame step (paper Sec. II frame conventions).

The viewing angles are checked against an explicit construction of the source
frame of the paper's basis equation (projecting the direction to the observer
onto it), and the polarisation-angle formula against the angle between the
wave-frame basis and the barycentre polarisation basis built from vectors.
"""
import math

import numpy as np
import pytest

from oracle.frame import frame_angles, to_ssb


def _unit(t, p):
    return np.array([math.sin(t) * math.cos(p), math.sin(t) * math.sin(p), math.cos(t)])


def _angles(seed):
    rng = np.random.default_rng(seed)
    return (math.acos(rng.uniform(-1, 1)), rng.uniform(0, 2 * math.pi),
            math.acos(rng.uniform(-1, 1)), rng.uniform(0, 2 * math.pi))


@pytest.mark.parametrize("seed", range(20))
def test_viewing_angles_from_the_source_frame_basis(seed):
    ts, ps, tk, pk = _angles(seed)
    R, S = _unit(ts, ps), _unit(tk, pk)
    n = math.sqrt(1 - np.dot(R, S) ** 2)
    x = np.cross(R, S) / n
    y = (R - np.dot(R, S) * S) / n
    z = S
    obs = -R                                  # from the source towards the observer
    theta = math.acos(np.dot(obs, z))
    phi = math.atan2(np.dot(obs, y), np.dot(obs, x))
    t_src, p_src, _ = frame_angles(ts, ps, tk, pk)
    assert abs(t_src - theta) < 1e-12
    assert abs(p_src - phi) < 1e-12 and abs(p_src + math.pi / 2) < 1e-15


@pytest.mark.parametrize("seed", range(20))
def test_polarisation_angle_from_the_wave_frame(seed):
    """tan psi = (y_w . p) / (-y_w . q) with the wave-frame y_w and the
    barycentre polarisation basis p = dR/dtheta_S, q = dR/dphi_S / sin theta_S."""
    ts, ps, tk, pk = _angles(100 + seed)
    R, S = _unit(ts, ps), _unit(tk, pk)
    yw = S - np.dot(S, R) * R
    yw /= np.linalg.norm(yw)
    p = np.array([math.cos(ts) * math.cos(ps), math.cos(ts) * math.sin(ps), -math.sin(ts)])
    q = np.array([-math.sin(ps), math.cos(ps), 0.0])
    psi_geo = math.atan2(np.dot(yw, p), -np.dot(yw, q))
    _, _, psi = frame_angles(ts, ps, tk, pk)
    # only 2 psi matters: compare e^{2 i psi}
    assert abs(np.exp(2j * psi) - np.exp(2j * psi_geo)) < 1e-12


def test_face_on_and_edge_on():
    t, p, psi = frame_angles(0.7, 1.1, 0.7, 1.1)          # R = S
    assert abs(t - math.pi) < 1e-7 and psi == 0.0
    ts, ps = 1.2, 0.3
    R = _unit(ts, ps)
    S = np.cross(R, [0.0, 0.0, 1.0])
    S /= np.linalg.norm(S)
    tk, pk = math.acos(S[2]), math.atan2(S[1], S[0])
    t, _, _ = frame_angles(ts, ps, tk, pk)                 # R . S = 0
    assert abs(t - math.pi / 2) < 1e-12


def test_rotation_is_unitary_and_composes():
    rng = np.random.default_rng(3)
    h = rng.standard_normal(50) + 1j * rng.standard_normal(50)
    assert np.allclose(np.abs(to_ssb(h, 0.37)), np.abs(h), rtol=1e-15)
    np.testing.assert_allclose(to_ssb(h, 0.0), -h, rtol=0, atol=0)
    two = to_ssb(to_ssb(h, 0.2), 0.5)
    np.testing.assert_allclose(two, np.exp(-2j * 0.7) * h, rtol=1e-14)
