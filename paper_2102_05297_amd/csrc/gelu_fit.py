"""Coefficients of gelu.h's tail polynomial: p(x) ~ log2 Phi(-x) on
[0, X] with X = kGeluTailMax, degree D, as a weighted least-squares fit in
the Chebyshev basis reweighted towards the largest errors (an approximation
of the minimax fit), expanded in powers of x and rounded to float32.

    python paper_2102_05297_amd/csrc/gelu_fit.py

prints the Horner lines of gelu_tail_log2 (highest power first) and the
largest error of the rounded polynomial in double precision; the float32
evaluation is checked by tests/gelu_check.cpp."""
import numpy as np
from numpy.polynomial import chebyshev as Ch
from numpy.polynomial import polynomial as Po
from scipy.special import log_ndtr

X, D = 6.0, 6


def main():
    x = np.linspace(0.0, X, 60001)
    y = log_ndtr(-x) / np.log(2.0)
    t = 2.0 * x / X - 1.0
    w = np.ones_like(x)
    for _ in range(80):
        c = Ch.chebfit(t, y, D, w=np.sqrt(w))
        err = Ch.chebval(t, c) - y
        w *= np.abs(err) / np.abs(err).max() + 1e-3
        w /= w.mean()
    # powers of t, then t = (2 / X) x - 1
    pt = Ch.cheb2poly(c)
    px = np.zeros(1)
    lin = np.array([-1.0, 2.0 / X])
    for k in range(len(pt) - 1, -1, -1):
        px = Po.polyadd(Po.polymul(px, lin), [pt[k]])
    p32 = px.astype(np.float32)
    e = np.abs(Po.polyval(x, p32.astype(np.float64)) - y).max()
    for k in range(D, -1, -1):
        print(f"{float(p32[k]):.9e}f")
    print(f"max |p - log2 Phi(-x)| on [0, {X}] (double evaluation): {e:.3e}")


if __name__ == "__main__":
    main()
