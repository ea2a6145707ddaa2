"""Oracle of the detector-frame step (paper Sec. II, the frame conventions after
Eq. (1)) -- test infrastructure only.

Sky position and spin direction in the solar-system-barycentre frame:
    R = (sin tS cos pS, sin tS sin pS, cos tS),  S = (sin tK cos pK, sin tK sin pK, cos tK).
The source frame has z along S and x along R x S, so the observer (direction
-R from the source) sits at the polar viewing angle cos(theta_src) = -R.S and
at azimuth phi_src = -pi/2.  The source-frame polarisation basis is turned by
pi/2 to align with the wave frame, a sign flip of h = h_plus - i h_cross.  The
barycentre frame follows by a rotation of the polarisation basis through the
polarisation angle psi, with
    tan psi = [cos tS sin tK cos(pS - pK) - sin tS cos tK] / [sin tK sin(pS - pK)].

Readings (the paper is garbled or silent here): psi is given by its tangent
(the printed formula lacks the tan); the rotation acts as
h_plus' = cos 2psi h_plus - sin 2psi h_cross, h_cross' = sin 2psi h_plus +
cos 2psi h_cross, i.e. h' = e^{-2 i psi} h, so the barycentre-frame waveform is
h_ssb = -e^{-2 i psi} h(theta_src, phi_src).  Only e^{2 i psi} enters, which the
tangent fixes without the branch of psi.  When R is parallel to S the angle is
undefined and psi = 0 is used.

Parity unpinned: the sense of the rotation (e^{-2 i psi} rather than
e^{+2 i psi}) is a convention the paper does not fix, so no test can pin it;
the viewing angles, psi itself and the unitarity of the rotation are pinned.
"""
from __future__ import annotations

import math

import numpy as np


def frame_angles(theta_s: float, phi_s: float, theta_k: float, phi_k: float):
    """(theta_src, phi_src, psi) from the sky and spin angles (module docstring)."""
    R = np.array([math.sin(theta_s) * math.cos(phi_s), math.sin(theta_s) * math.sin(phi_s),
                  math.cos(theta_s)])
    S = np.array([math.sin(theta_k) * math.cos(phi_k), math.sin(theta_k) * math.sin(phi_k),
                  math.cos(theta_k)])
    c = float(np.dot(R, S))
    theta_src = math.acos(max(-1.0, min(1.0, -c)))
    num = (math.cos(theta_s) * math.sin(theta_k) * math.cos(phi_s - phi_k)
           - math.sin(theta_s) * math.cos(theta_k))
    den = math.sin(theta_k) * math.sin(phi_s - phi_k)
    psi = math.atan2(num, den) if (num != 0.0 or den != 0.0) else 0.0
    return theta_src, -math.pi / 2, psi


def to_ssb(h: np.ndarray, psi: float) -> np.ndarray:
    """Barycentre-frame waveform from the source-frame one: -e^{-2 i psi} h."""
    return -np.exp(-2j * psi) * np.asarray(h, dtype=np.complex128)
