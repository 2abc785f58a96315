"""Derive the FIT reading of q(sigma) from the oracle (run by hand; prints constants).

For each target width sigma, q*(sigma) minimises the mass-normalised shape error
  E(q) = || h_q/sum(h_q) - g/sum(g) ||_2 / || g/sum(g) ||_2
between the impulse response h_q of one causal + anti-causal 3rd-RF pass built
with the Theorem 3.1 polynomials at q (mode LITERAL with sigma := q; beta only
scales h and drops out of E) and the Gaussian g(x) = exp(-x^2/(2 sigma^2)) of
Appendix A, eq. "convolution".  The minimisers are then fitted by
  q(sigma) = sigma - F0 + F1/(sigma + F2).
Only the oracle is called.  Usage: python -m oracle.fit_q
"""
import numpy as np
from scipy.optimize import minimize_scalar, least_squares

import oracle


def impulse(q, m):
    P = oracle.Problem(np.ones((1, m)), np.full((1, m), q), np.full((1, m), q))
    x = np.zeros((1, m))
    x[0, m // 2] = 1.0
    return P.apply_dir(x, "x")[0]


def shape_error(h, sigma):
    m = h.size
    i = np.arange(m) - m // 2
    g = np.exp(-i * i / (2.0 * sigma * sigma))
    hn, gn = h / h.sum(), g / g.sum()
    return np.linalg.norm(hn - gn) / np.linalg.norm(gn)


def q_star(sigma):
    m = int(60 * sigma) | 1
    r = minimize_scalar(lambda q: shape_error(impulse(q, m), sigma),
                        bounds=(0.2 * sigma, 1.2 * sigma + 1), method="bounded",
                        options={"xatol": 1e-7})
    return r.x, r.fun


def main():
    sig = np.array([1.5, 2, 2.5, 3, 4, 5, 6, 8, 10, 12, 14, 16], float)
    qs = np.array([q_star(s)[0] for s in sig])
    for s, q in zip(sig, qs):
        print(f"sigma {s:5.2f}  q* {q:.6f}")
    res = least_squares(lambda f: sig - f[0] + f[1] / (sig + f[2]) - qs, x0=[1.0, 0.3, -0.3])
    f0, f1, f2 = res.x
    print(f"FIT_F0 = {f0:.7f}\nFIT_F1 = {f1:.7f}\nFIT_F2 = {f2:.7f}")
    print("max |fit - q*| =", np.abs(sig - f0 + f1 / (sig + f2) - qs).max())


if __name__ == "__main__":
    main()
