"""Plain CPU oracle for the 2-D five-point Jacobi (Laplace) sweep.

TEST INFRASTRUCTURE. Only the test suite, the smoke check and the benchmark's
CPU-baseline leg may use this module. It shares no code with the GPU library.

What the method computes (listing of the 2-D Laplace solver, Section III-A):
two same-shape arrays carry the same boundary ring; each iteration writes the
interior of the second array from the first,

    u2[1:-1,1:-1] = 0.25 * (u1[:-2,1:-1] + u1[2:,1:-1] + u1[1:-1,:-2] + u1[1:-1,2:])

and then swaps the two names. The right-hand side reads only the other array
(Section III-A: an assignment whose right side depends on its own output is
rejected, which is why two arrays are used). Python evaluates the sum left to
right, so each interior point is c*(((N + S) + W) + E) with N = row above,
S = row below, W = column to the left, E = column to the right, then one
multiply. The boundary ring is never written.

Readings where the paper is silent (each is listed with its reason in the
design notes):
* precision: FP64 (NumPy's default; the paper states none);
* one input u0 whose ring both buffers carry; the output is the whole grid;
* grids with fewer than 3 rows or columns have an empty interior, so the
  output equals the input (NumPy's empty-slice semantics);
* a general coefficient c replaces the listing's 0.25 (c = 0.25 by default).

Everything here is a direct transcription of those definitions into NumPy
slicing, with no blocking, fusion or reordering.
"""

from __future__ import annotations

import numpy as np

__all__ = [
    "sweep",
    "jacobi5",
    "jacobi5_states",
    "sweep_adjoint",
    "jacobi5_adjoint",
    "grad_c",
    "abs_reference",
    "gamma",
    "bound_fp32",
    "bound_adjoint_fp32",
    "bound_hilo_from_abs",
    "bound_grad_c_fp32",
    "hilo_delta",
    "hilo_encode",
    "hilo_decode",
    "bound_hilo",
    "HILO_QBITS",
    "hilo_sweep_model",
    "jacobi5_hilo_model",
    "error_report",
]


# ---------------------------------------------------------------------------
# Forward method (listing of the Laplace solver, Section III-A)
# ---------------------------------------------------------------------------

def sweep(src: np.ndarray, dst: np.ndarray, c=0.25) -> None:
    """One Jacobi sweep: dst's interior from src, dst's ring untouched.

    Written exactly as the listing's loop body (Section III-A), with the
    coefficient 0.25 generalised to c. NumPy evaluates the sum left to right,
    elementwise, in the arrays' precision, with one rounding per operation.
    """
    if src.shape[0] < 3 or src.shape[1] < 3:
        return  # empty interior: the slices are empty
    dst[1:-1, 1:-1] = c * (src[:-2, 1:-1] + src[2:, 1:-1] + src[1:-1, :-2] + src[1:-1, 2:])


def jacobi5(u0, T: int, c=0.25, dtype=np.float64) -> np.ndarray:
    """u after T sweeps with a ping-pong swap, from initial grid u0.

    Both buffers start as copies of u0, so both carry u0's boundary ring (the
    listing fills the same ring into both arrays, Section III-A). After each
    sweep the names swap; the result is the last-written buffer (named u1
    after the swap in the listing). T = 0 returns a copy of u0.
    """
    if T < 0:
        raise ValueError("T must be >= 0")
    a = np.array(u0, dtype=dtype, copy=True)
    b = a.copy()
    if dtype == np.float32:
        c = np.float32(c)
    for _ in range(T):
        sweep(a, b, c)
        a, b = b, a
    return a


def jacobi5_states(u0, T: int, c=0.25, dtype=np.float64) -> list[np.ndarray]:
    """The list [u_0, u_1, ..., u_T] of all intermediate grids of `jacobi5`."""
    a = np.array(u0, dtype=dtype, copy=True)
    if dtype == np.float32:
        c = np.float32(c)
    states = [a.copy()]
    for _ in range(T):
        b = a.copy()
        sweep(a, b, c)
        a = b
        states.append(a.copy())
    return states


# ---------------------------------------------------------------------------
# Adjoint (transpose of the sweep). Not in the paper: the gradient extension.
# ---------------------------------------------------------------------------

def sweep_adjoint(g: np.ndarray, c=0.25) -> np.ndarray:
    """S^T g, where S is the linear map of one sweep (ring copied, interior averaged).

    By the definition of the transpose, (S^T g)[n] = sum over m of S[m, n] g[m]:
    every ring point m passes g[m] to itself with weight 1, and every interior
    point m passes c * g[m] to each of its four neighbours (the points its
    forward update reads). Written here in that scatter form.
    """
    H, W = g.shape
    out = np.array(g, dtype=np.float64, copy=True)
    if H < 3 or W < 3:
        return out  # S is the identity
    gi = np.array(g[1:-1, 1:-1], dtype=np.float64)
    out[1:-1, 1:-1] = 0.0          # interior points have no identity term
    out[:-2, 1:-1] += c * gi       # forward update of (i, j) reads (i-1, j)
    out[2:, 1:-1] += c * gi        # ... reads (i+1, j)
    out[1:-1, :-2] += c * gi       # ... reads (i, j-1)
    out[1:-1, 2:] += c * gi        # ... reads (i, j+1)
    return out


def jacobi5_adjoint(w, T: int, c=0.25) -> np.ndarray:
    """dL/du0 for L = sum(w * jacobi5(u0, T, c)): apply S^T to w, T times, in FP64."""
    g = np.array(w, dtype=np.float64, copy=True)
    for _ in range(T):
        g = sweep_adjoint(g, c)
    return g


def grad_c(u0, w, T: int, c=0.25) -> float:
    """dL/dc for L = sum(w * jacobi5(u0, T, c)), in FP64.

    With u_{k+1} = S_c(u_k) and lam_k = dL/du_k (lam_T = w,
    lam_k = S^T lam_{k+1}), the chain rule gives
    dL/dc = sum_k sum_{interior m} lam_{k+1}[m] * (d/dc S_c(u_k))[m], and the
    derivative of an interior update c*nbrsum is nbrsum(u_k)[m].
    """
    states = jacobi5_states(u0, T, c)
    lam = np.array(w, dtype=np.float64, copy=True)
    total = 0.0
    H, W = lam.shape
    for k in range(T - 1, -1, -1):
        if H >= 3 and W >= 3:
            u = states[k]
            nbrsum = u[:-2, 1:-1] + u[2:, 1:-1] + u[1:-1, :-2] + u[1:-1, 2:]
            total += float(np.sum(lam[1:-1, 1:-1] * nbrsum))
        lam = sweep_adjoint(lam, c)
    return total


# ---------------------------------------------------------------------------
# Error bounds (floating-point analysis of the forward sweep)
# ---------------------------------------------------------------------------

def abs_reference(u0, T: int, c=0.25) -> np.ndarray:
    """|J| |u0| where J is the linear map of T sweeps; used to scale error bounds.

    All weights of a sweep are nonnegative when c >= 0, so |J| |u0| is the
    method itself applied to |u0| with |c|.
    """
    return jacobi5(np.abs(np.asarray(u0, dtype=np.float64)), T, abs(float(c)))


def gamma(k: int, u: float) -> float:
    """gamma_k = k u / (1 - k u), the standard bound for k rounded operations."""
    return k * u / (1.0 - k * u)


def bound_fp32(u0, T: int, c=0.25) -> np.ndarray:
    """Componentwise bound on |y32 - y64| after T FP32 sweeps from FP32-exact u0.

    One FP32 sweep adds three numbers (error <= gamma_3 times the sum of
    magnitudes) and multiplies by c (exact when c is a power of two; otherwise
    one more rounding plus the rounding of c itself, hence gamma_5). Errors of
    earlier sweeps pass through later ones with the nonnegative weights of |S|,
    so after T sweeps |err| <= T * g * (1 + g)^T * (|J| |u0|).
    """
    u = 2.0 ** -24
    cf = float(c)
    exact_c = cf != 0.0 and np.float32(cf) == cf and np.frexp(abs(cf))[0] == 0.5
    g = gamma(3, u) if exact_c else gamma(5, u)
    return T * g * (1.0 + g) ** T * abs_reference(u0, T, c)


def bound_adjoint_fp32(w, T: int, c=0.25) -> np.ndarray:
    """Componentwise bound on |g32 - g64| after T FP32 transposed sweeps of FP32-exact w.

    One transposed sweep adds at most four neighbour terms (three additions),
    multiplies by c (exact for a power of two) and, on the ring, adds the
    point's own value: at most gamma_4 (gamma_5 for a general c) times the sum
    of the magnitudes combined, i.e. of |S^T| |g|. As for the forward method,
    |err| <= T g (1 + g)^T (|J|^T |w|), and |J|^T |w| is the adjoint applied to
    |w| with |c| (all weights nonnegative).
    """
    u = 2.0 ** -24
    cf = float(c)
    m, _ = np.frexp(abs(cf))
    g = gamma(4, u) if (cf != 0.0 and m == 0.5) else gamma(5, u)
    return T * g * (1.0 + g) ** T * jacobi5_adjoint(np.abs(np.asarray(w, dtype=np.float64)), T, abs(cf))


def bound_grad_c_fp32(u0, w, T: int, c=0.25) -> float:
    """Bound on |dL/dc (FP32 forward states + FP32 adjoint, FP64 dot) - dL/dc (FP64)|.

    Per step k the computed term is sum_m lam^_{k+1}[m] * nbrsum^_k[m] with
    |lam^_{k+1} - lam_{k+1}| <= G_{k+1} (bound_adjoint_fp32 after T-k-1 steps)
    and |nbrsum^_k - nbrsum(u_k)| <= E_k = nbrsum(F_k) + gamma_3 nbrsum(|u_k| + F_k),
    F_k = bound_fp32(u0, k) the forward state error; so the step's error is at
    most sum_m G_{k+1} (|nbrsum(u_k)| + E_k) + |lam_{k+1}| E_k. The FP64
    products and sums add a relative 2^-40 of the sum of magnitudes.
    """
    u0 = np.asarray(u0, dtype=np.float64)
    w = np.asarray(w, dtype=np.float64)
    H, W = u0.shape
    if H < 3 or W < 3 or T == 0:
        return 0.0
    g3 = gamma(3, 2.0 ** -24)
    states = jacobi5_states(u0, T, c)
    lams = [None] * (T + 1)
    lams[T] = w.copy()
    for k in range(T - 1, -1, -1):
        lams[k] = sweep_adjoint(lams[k + 1], c)

    def nsum(a):
        return a[:-2, 1:-1] + a[2:, 1:-1] + a[1:-1, :-2] + a[1:-1, 2:]

    total = 0.0
    mag = 0.0
    for k in range(T):
        F = bound_fp32(u0, k, c)
        au = np.abs(states[k])
        E = nsum(F) + g3 * nsum(au + F)
        G = bound_adjoint_fp32(w, T - k - 1, c)[1:-1, 1:-1]
        lam = np.abs(lams[k + 1][1:-1, 1:-1])
        ns = np.abs(nsum(states[k]))
        total += float(np.sum(G * (ns + E) + lam * E))
        mag += float(np.sum((lam + G) * (ns + E)))
    return total + 2.0 ** -40 * mag


# ---------------------------------------------------------------------------
# hi/lo encoding for the reduced-precision form (not in the paper)
# ---------------------------------------------------------------------------

HILO_QBITS = 16  # lo is an int16 count of units 2^-16 * ulp32(hi)


def hilo_delta(hi: np.ndarray) -> np.ndarray:
    """Quantum of the lo part: 2^(e - 23 - 16), floored at 2^-149.

    e is the unbiased exponent that sets the FP32 unit in the last place of hi
    (for zero and subnormal hi the exponent of the smallest normal, -126), so
    2^(e-23) = ulp32(hi) and the quantum is ulp32(hi) * 2^-16.
    """
    hi = np.asarray(hi, dtype=np.float32)
    biased = ((hi.view(np.uint32) >> 23) & 0xFF).astype(np.int64)
    e = np.maximum(biased, 1) - 127
    return np.ldexp(1.0, np.maximum(e - 23 - HILO_QBITS, -149))


def hilo_encode(x):
    """FP64 x -> (hi FP32, q int16) with x ~ hi + q * delta(hi).

    hi = RN32(x) and q = rint((x - hi) / delta) (round half to even). x - hi is
    exact in FP64 and delta is a power of two, so rint is the only rounding.
    Since |x - hi| <= ulp32(hi)/2, q lies in [-32768, 32768]; the one value
    int16 cannot hold, +32768, is renormalised exactly: hi steps up to the
    next FP32 number and q is recomputed from the (now negative) remainder,
    which lands in [-32768, -16384]. So |x - decode| <= delta/2 always.
    """
    x = np.asarray(x, dtype=np.float64)
    with np.errstate(over="ignore"):
        hi = x.astype(np.float32)
    if not np.all(np.isfinite(hi)):
        raise ValueError("hi/lo encoding needs |x| below the FP32 range")
    q = np.rint((x - hi.astype(np.float64)) / hilo_delta(hi))
    over = q > 32767
    if np.any(over):
        hi = hi.copy()
        hi[over] = np.nextafter(hi[over], np.float32(np.inf))
        q[over] = np.rint((x[over] - hi[over].astype(np.float64)) / hilo_delta(hi[over]))
    assert np.all(q >= -32768) and np.all(q <= 32767)
    return hi, q.astype(np.int16)


def hilo_decode(hi, q) -> np.ndarray:
    """(hi, q) -> FP64 hi + q * delta(hi); exact in FP64."""
    hi = np.asarray(hi, dtype=np.float32)
    return hi.astype(np.float64) + np.asarray(q, dtype=np.float64) * hilo_delta(hi)


def bound_hilo(u0, T: int, c=0.25) -> np.ndarray:
    """Componentwise bound on |y - y64| for the hi/lo form after T sweeps.

    Encoding the input and re-quantising after each sweep each perturb a value
    v by at most half a quantum, delta/2 <= 2^-40 |hi| <= 2^-40 (1 + 2^-22) |v|.
    The FP32 arithmetic of one sweep is exact up to the recursive sums of the
    low parts: four lo terms (each <= 2^-24 |h|) and three TwoSum errors (each
    <= 2^-24 times a partial sum), so at most about 17 * 2^-48 times the sum
    of the neighbour magnitudes; a general c adds a double-word product
    (20 * 2^-48 in all). These perturbations pass through later sweeps with the
    weights of |S|, so
    |err| <= ((T + 1) 2^-40 (1 + 2^-22) + T a) (1 + 2^-39)^T (|J| |u0|), a as above,
    plus an absolute term for values whose quantum is floored at 2^-149.
    """
    return bound_hilo_from_abs(abs_reference(u0, T, c), T, c)


def bound_hilo_from_abs(absref, T: int, c=0.25) -> np.ndarray:
    """bound_hilo given |J| |u0| (abs_reference) computed elsewhere, e.g. by the C twin."""
    cf = float(c)
    m, _ = np.frexp(abs(cf))
    a = 17 * 2.0 ** -48 if (cf != 0.0 and m == 0.5) else 20 * 2.0 ** -48
    per = (T + 1) * 2.0 ** -40 * (1.0 + 2.0 ** -22) + T * a
    return per * (1.0 + 2.0 ** -39) ** T * np.asarray(absref, dtype=np.float64) + (T + 1) * 2.0 ** -149


# ---------------------------------------------------------------------------
# Bit-level model of the hi/lo sweep (its steps in order, NumPy float32)
# ---------------------------------------------------------------------------

def _delta_exp32(h: np.ndarray) -> np.ndarray:
    """k with delta(h) = 2^k, from the FP32 exponent field of h (see hilo_delta)."""
    E = ((np.asarray(h, dtype=np.float32).view(np.uint32) >> 23) & 0xFF).astype(np.int32)
    return np.maximum(np.maximum(E, 1) - 127 - 23 - HILO_QBITS, -149).astype(np.int32)


def _two_sum(a: np.ndarray, b: np.ndarray):
    """Knuth's TwoSum in FP32: s = fl(a + b) and e with s + e == a + b exactly."""
    s = a + b
    bb = s - a
    e = (a - (s - bb)) + (b - bb)
    return s, e


def _hilo_requantise(H: np.ndarray, L: np.ndarray):
    """(H, L) with |L| <= ulp(H)/2 -> (hi, q); q = +32768 moves one ulp into hi."""
    k = _delta_exp32(H)
    qf = np.rint(np.ldexp(L, -k)).astype(np.float32)
    over = qf > 32767
    if np.any(over):
        H = H.copy()
        L = L.copy()
        ulp = np.ldexp(np.float32(1.0), k[over] + 16).astype(np.float32)
        H[over] = H[over] + ulp
        L[over] = L[over] - ulp
        k2 = _delta_exp32(H[over])
        qf[over] = np.rint(np.ldexp(L[over], -k2)).astype(np.float32)
    return H, qf.astype(np.int16)


def hilo_sweep_model(hi: np.ndarray, q: np.ndarray, c=0.25):
    """One sweep of the hi/lo form on an encoded grid, step by step in FP32.

    decode each point to (h, l = q * delta(h)); for each interior point,
    s1,e1 = TwoSum(N.h, S.h); s2,e2 = TwoSum(s1, W.h); s3,e3 = TwoSum(s2, E.h);
    low = (((N.l + S.l) + W.l) + E.l) + ((e1 + e2) + e3); (H, L) = TwoSum(s3, low);
    scale by c (exact for a power of two, else a double-word product using the
    exact FP32 product error); re-encode. The ring is unchanged.
    """
    hi = np.asarray(hi, dtype=np.float32)
    q = np.asarray(q, dtype=np.int16)
    out_h = hi.copy()
    out_q = q.copy()
    if hi.shape[0] < 3 or hi.shape[1] < 3:
        return out_h, out_q
    lo = np.ldexp(q.astype(np.float32), _delta_exp32(hi)).astype(np.float32)
    nh, sh, wh, eh = hi[:-2, 1:-1], hi[2:, 1:-1], hi[1:-1, :-2], hi[1:-1, 2:]
    nl, sl, wl, el = lo[:-2, 1:-1], lo[2:, 1:-1], lo[1:-1, :-2], lo[1:-1, 2:]
    s1, e1 = _two_sum(nh, sh)
    s2, e2 = _two_sum(s1, wh)
    s3, e3 = _two_sum(s2, eh)
    low = (((nl + sl) + wl) + el) + ((e1 + e2) + e3)
    H, L = _two_sum(s3, low)
    cf = float(c)
    c_hi = np.float32(cf)
    c_lo = np.float32(cf - float(c_hi))
    m, _ = np.frexp(abs(cf))
    if cf != 0.0 and m == 0.5 and c_lo == 0:
        H = H * c_hi
        L = L * c_hi
    else:
        p = H * c_hi
        # exact error of the FP32 product: H*c_hi has 48 bits, exact in FP64
        ep = (H.astype(np.float64) * np.float64(c_hi) - p.astype(np.float64)).astype(np.float32)
        ep = ep + (H * c_lo + L * c_hi)
        H = p + ep
        L = ep - (H - p)
    Hn, qn = _hilo_requantise(H.astype(np.float32), L.astype(np.float32))
    out_h[1:-1, 1:-1] = Hn
    out_q[1:-1, 1:-1] = qn
    return out_h, out_q


def jacobi5_hilo_model(u0, T: int, c=0.25) -> np.ndarray:
    """FP64 result of the hi/lo form: encode u0, T model sweeps, decode; ring copied from u0."""
    u0 = np.asarray(u0, dtype=np.float64)
    hi, q = hilo_encode(u0)
    for _ in range(T):
        hi, q = hilo_sweep_model(hi, q, c)
    out = hilo_decode(hi, q)
    if u0.shape[0] >= 1 and u0.shape[1] >= 1:
        out[0, :] = u0[0, :]
        out[-1, :] = u0[-1, :]
        out[:, 0] = u0[:, 0]
        out[:, -1] = u0[:, -1]
    return out


def error_report(y, y_ref, absref) -> dict:
    """Errors of y against y_ref: normwise, componentwise (vs |J||u0|) and raw relative.

    * normwise: max |y - y*| / max |y*|
    * componentwise: max over points of |y - y*| / (|J| |u0|) (points where the
      scale is zero must match exactly)
    * relative: max |y - y*| / |y*| over points with |y*| >= 1e-3 max |y*|
    """
    y = np.asarray(y, dtype=np.float64)
    y_ref = np.asarray(y_ref, dtype=np.float64)
    absref = np.asarray(absref, dtype=np.float64)
    err = np.abs(y - y_ref)
    scale = np.max(np.abs(y_ref)) if y_ref.size else 0.0
    normwise = float(np.max(err) / scale) if scale > 0 else float(np.max(err, initial=0.0))
    nz = absref > 0
    comp = float(np.max(err[nz] / absref[nz], initial=0.0))
    comp_zero_ok = bool(np.all(err[~nz] == 0))
    big = np.abs(y_ref) >= 1e-3 * scale
    rel = float(np.max(err[big] / np.abs(y_ref[big]), initial=0.0)) if scale > 0 else 0.0
    return {
        "normwise": normwise,
        "componentwise": comp,
        "componentwise_zero_ok": comp_zero_ok,
        "relative_large": rel,
        "max_abs": float(np.max(err, initial=0.0)),
    }
