"""View-dependent colour c_i(d) as real spherical harmonics, FP64 (test infrastructure only).

Sec. 3 leaves the colour model to 4DGS; this build uses RGB real SH up to
degree 3.  The basis is derived here from SciPy's complex spherical harmonics
(which carry the Condon-Shortley phase), not from hand-typed polynomials:

    k = l*l + l + m,   m = -l..l
    m > 0:  sqrt(2) * Re Y_l^m(d)
    m = 0:            Y_l^0(d)
    m < 0:  sqrt(2) * Im Y_l^{|m|}(d)

Colour = max(0, sum_k sh_k Y_k(d) + 0.5), d the unit vector from the camera
centre to the (conditional) Gaussian mean.
"""
from __future__ import annotations

import numpy as np
from scipy.special import sph_harm_y


def real_sh_basis(d: np.ndarray, degree: int = 3) -> np.ndarray:
    """d: (n, 3) unit vectors -> (n, (degree+1)^2) basis values."""
    d = np.asarray(d, dtype=np.float64)
    polar = np.arccos(np.clip(d[:, 2], -1.0, 1.0))
    azim = np.arctan2(d[:, 1], d[:, 0])
    out = np.empty((d.shape[0], (degree + 1) ** 2))
    for l in range(degree + 1):
        for m in range(-l, l + 1):
            Y = sph_harm_y(l, abs(m), polar, azim)
            if m > 0:
                val = np.sqrt(2.0) * Y.real
            elif m == 0:
                val = Y.real
            else:
                val = np.sqrt(2.0) * Y.imag
            out[:, l * l + l + m] = val
    return out


def sh_color(sh_rows: np.ndarray, d: np.ndarray, degree: int = 3) -> np.ndarray:
    """sh_rows: (n, 16, 3) coefficients; d: (n, 3) unit directions -> (n, 3) rgb."""
    k = (degree + 1) ** 2
    Y = real_sh_basis(d, degree)
    raw = np.einsum('nk,nkc->nc', Y, sh_rows[:, :k, :]) + 0.5
    return np.maximum(raw, 0.0)
