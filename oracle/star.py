"""CPU oracle for general constant-coefficient star stencils (test infrastructure).

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module. It shares no code with the GPU library.

The paper's frontend turns any slice assignment into a generated kernel
(Section III-B and III-C): the ghost depth is the largest index offset the
expression reads, and assignments of the same output shape with no path
between them may be fused into one kernel (node fusion, Section III-B). This
module defines the general star stencil of radius R written as such a slice
expression, evaluated left to right:

    out[R:-R, R:-R] = c0*A[c] + cN1*A[N1] + cS1*A[S1] + cW1*A[W1] + cE1*A[E1]
                              + cN2*A[N2] + ... + cER*A[ER]

where Nk/Sk/Wk/Ek are the slices shifted k rows up/down or k columns left/right.
Every product is rounded, then added to the running sum (no fused
multiply-add). The frame of width R is never written. Grids with fewer than
2R+1 rows or columns have nothing to update.
"""

from __future__ import annotations

import numpy as np

__all__ = ["StarCoef", "star_apply", "star_iterate", "star_lambda"]


class StarCoef:
    """Coefficients of a radius-R star stencil: c0 and cn/cs/cw/ce[k-1] for k = 1..R."""

    def __init__(self, c0, cn, cs, cw, ce):
        self.c0 = float(c0)
        self.cn = [float(v) for v in cn]
        self.cs = [float(v) for v in cs]
        self.cw = [float(v) for v in cw]
        self.ce = [float(v) for v in ce]
        R = len(self.cn)
        if not (len(self.cs) == len(self.cw) == len(self.ce) == R) or not 1 <= R <= 4:
            raise ValueError("radius must be 1..4 with four coefficient lists of that length")
        self.R = R

    @staticmethod
    def jacobi(c=0.25):
        """The five-point Laplace sweep written as a star stencil (c*N + c*S + c*W + c*E)."""
        return StarCoef(0.0, [c], [c], [c], [c])


def star_apply(A, coef: StarCoef, dtype=np.float64) -> np.ndarray:
    """One application: a copy of A whose depth-R interior is the star stencil of A."""
    A = np.asarray(A, dtype=dtype)
    out = A.copy()
    R = coef.R
    H, W = A.shape
    if H < 2 * R + 1 or W < 2 * R + 1:
        return out

    def sl(di, dj):
        return A[R + di:H - R + di, R + dj:W - R + dj]

    t = dtype
    acc = t(coef.c0) * sl(0, 0)
    for k in range(1, R + 1):
        acc = acc + t(coef.cn[k - 1]) * sl(-k, 0)
        acc = acc + t(coef.cs[k - 1]) * sl(k, 0)
        acc = acc + t(coef.cw[k - 1]) * sl(0, -k)
        acc = acc + t(coef.ce[k - 1]) * sl(0, k)
    out[R:H - R, R:W - R] = acc
    return out


def star_iterate(u0, T: int, coef: StarCoef, dtype=np.float64) -> np.ndarray:
    """T applications with a ping-pong swap (both buffers start as u0, so the frame stays u0's)."""
    a = np.array(u0, dtype=dtype, copy=True)
    for _ in range(T):
        a = star_apply(a, coef, dtype)
    return a


def star_lambda(coef: StarCoef, a: float, b: float) -> float:
    """Symbol of a star stencil with cn = cs, cw = ce on sin(a i) sin(b j):
    c0 + sum_k 2 cn_k cos(k a) + 2 cw_k cos(k b)."""
    lam = coef.c0
    for k in range(1, coef.R + 1):
        lam += 2 * coef.cn[k - 1] * np.cos(k * a) + 2 * coef.cw[k - 1] * np.cos(k * b)
    return lam
