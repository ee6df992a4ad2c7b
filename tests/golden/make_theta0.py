"""Least-squares fit of the 8-parameter ansatz to the plasma and MPA terms.

f_theta(x) = [sum_p th_p x^p + i sum_p th_{4+p} x^p] / (1 + x^4), x = I/I_a
(stand-in for the effective-lens function of Eq. (6) and (9)).  The real part
is fitted to the saturating plasma index -x^K/(1+x^(K-1)) (Eq. (3), plasma
term); the imaginary part to the small-step MPA attenuation exponent
x^(K-1)/2 (Eq. (3), absorption term, with beta_K I_a^(K-1) = k0 n2 I_a), on
1001 points of x in [0, 1] (I up to I_a; a wider range makes the imaginary
fit ill-conditioned, with coefficients in the hundreds).  Prints the vector that ``workloads.THETA0``
holds; ``tests/test_oracle_pins.py`` re-runs the fit and compares.
"""
import numpy as np


def fit_theta0(order: int = 8):
    x = np.linspace(0.0, 1.0, 1001)
    den = 1.0 + x ** 4
    basis = np.stack([x ** p / den for p in range(1, 5)], axis=1)
    re_t = -x ** order / (1.0 + x ** (order - 1))
    im_t = 0.5 * x ** (order - 1)
    th_re = np.linalg.lstsq(basis, re_t, rcond=None)[0]
    th_im = np.linalg.lstsq(basis, im_t, rcond=None)[0]
    return np.concatenate([th_re, th_im])


if __name__ == "__main__":
    print(", ".join("%.8g" % v for v in fit_theta0()))
