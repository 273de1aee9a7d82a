"""Lazy NumPy-like frontend: slice assignments become a DAG of kernels (Section III-B).

This is the paper's programming model on top of libsten, for one GPU::

    ctx = Context(max_depth=64)
    u1 = ctx.create_array((H, W)); u2 = ctx.create_array((H, W))
    u1[0, :] = u1[-1, :] = u1[:, 0] = u1[:, -1] = 1
    u2[0, :] = u2[-1, :] = u2[:, 0] = u2[:, -1] = 1
    for _ in range(10):
        u2[1:-1, 1:-1] = 0.25 * (u1[:-2, 1:-1] + u1[2:, 1:-1] + u1[1:-1, :-2] + u1[1:-1, 2:])
        u1, u2 = u2, u1
    ctx.sync(); result = u1.tensor()

What it does, following Section III-A/III-B of the paper:

* every assignment to an array slice records the right side as an expression
  tree (AST) over same-shape slices of other arrays, scalars, +, -, *, /,
  unary minus and ``** 2``; the tree is parameterised (arrays are
  placeholders), so iterations that only swap arrays share one AST;
* an assignment whose right side reads the array it writes is rejected
  (``InPlaceDependencyError``), which is why the listing uses two arrays;
* nodes form a DAG with true, anti and output dependencies tracked per array
  (conservative: per array, not per index);
* the DAG is sent to the backend when ``sync()`` is called or when its depth
  would exceed ``max_depth``; kernel launches are asynchronous, so the Python
  side keeps building the next DAG while the GPU executes the previous one
  (pipelining);
* before execution, consecutive nodes with the same output region and no path
  between them are fused (node fusion);
* a run of consecutive Jacobi nodes over the whole interior that ping-pong
  between two arrays (the listing's loop) runs as one chain of blocked
  launches (several iterations per pass over HBM) when both arrays' boundary
  rings are known to hold the same values. The frontend knows a ring from the
  fill nodes that wrote it (arrays start as zeros); any other write to a ring,
  ``Context.invalidate(array)``, or ``Array.tensor()`` (which hands the data
  out) makes it unknown. Both arrays end as after one node at a time.

Backend: recognised ASTs map to hand-written libsten kernels - scalar fills
-> ``sten_fill_rect_f64``; the listing's update ``c*(N + S + W + E)`` on any
rectangle -> ``sten_sweep_f64`` on a view; a left-to-right sum of
``coef * shifted slice`` terms in the canonical star order ->
``sten_star_f64`` (fused nodes that read the same array share one launch).
Every other AST, and every fused group of them, becomes a generated kernel
(``sten_expr_run``: libsten emits HIP source for the group, compiles it at run
time and launches one thread per two adjacent output elements), as the paper's
backend does for all ASTs (Section III-C).
"""

from __future__ import annotations

import ctypes
import itertools
import struct
from dataclasses import dataclass, field

__all__ = ["Context", "Array", "InPlaceDependencyError"]


class InPlaceDependencyError(ValueError):
    """The right side of an assignment reads the array being assigned."""


# ---------------------------------------------------------------------------
# Expressions
# ---------------------------------------------------------------------------

class Expr:
    __slots__ = ()

    def __add__(self, o):
        return BinOp("+", self, _wrap(o))

    def __radd__(self, o):
        return BinOp("+", _wrap(o), self)

    def __sub__(self, o):
        return BinOp("-", self, _wrap(o))

    def __rsub__(self, o):
        return BinOp("-", _wrap(o), self)

    def __mul__(self, o):
        return BinOp("*", self, _wrap(o))

    def __rmul__(self, o):
        return BinOp("*", _wrap(o), self)

    def __truediv__(self, o):
        return BinOp("/", self, _wrap(o))

    def __rtruediv__(self, o):
        return BinOp("/", _wrap(o), self)

    def __neg__(self):
        return Unary("neg", self)

    def __pos__(self):
        return self

    def __pow__(self, k):
        # NumPy computes x ** 2 as x * x (one rounding); other powers are not supported
        if isinstance(k, (int, float)) and float(k) == 2.0:
            return Unary("sq", self)
        raise NotImplementedError("only ** 2 is supported")


@dataclass(eq=False, slots=True)
class Const(Expr):
    value: float


@dataclass(eq=False, slots=True)
class Ref(Expr):
    array: "Array"
    region: tuple  # (r0, r1, c0, c1), half-open, step 1


@dataclass(eq=False, slots=True)
class BinOp(Expr):
    op: str
    a: Expr
    b: Expr


@dataclass(eq=False, slots=True)
class Unary(Expr):
    op: str  # "neg" or "sq"
    a: Expr


def _wrap(v):
    if isinstance(v, Expr):
        return v
    if isinstance(v, (int, float)):
        return Const(float(v))
    raise TypeError(f"unsupported operand {type(v).__name__}")


def _norm(s, n: int) -> tuple[int, int]:
    if isinstance(s, int):
        i = s + n if s < 0 else s
        if not 0 <= i < n:
            raise IndexError("index out of range")
        return i, i + 1
    if isinstance(s, slice):
        start, stop, step = s.indices(n)
        if step != 1:
            raise NotImplementedError("strided views are not supported (Section III-D)")
        return start, max(start, stop)
    raise TypeError("indices must be ints or slices")


_REGION_TEXT: dict = {}


def _walk(e: Expr, names: dict, refs: list) -> str:
    """One pass over an expression: collects its slice references in order and returns the
    parameterised AST text (arrays become placeholders A0, A1, ... in order of first use)."""
    t = type(e)
    if t is Ref:
        refs.append(e)
        k = names.get(e.array.uid)
        if k is None:
            k = names[e.array.uid] = f"A{len(names)}"
        rt = _REGION_TEXT.get(e.region)
        if rt is None:
            if len(_REGION_TEXT) > 65536:
                _REGION_TEXT.clear()
            rt = _REGION_TEXT[e.region] = f"[{e.region}]"
        return k + rt
    if t is BinOp:
        return f"({_walk(e.a, names, refs)}{e.op}{_walk(e.b, names, refs)})"
    if t is Const:
        return repr(e.value)
    return f"{e.op}({_walk(e.a, names, refs)})"


# ---------------------------------------------------------------------------
# Arrays and DAG nodes
# ---------------------------------------------------------------------------

_uids = itertools.count()

# An array's boundary ring in 8 parts: 4 corners, then the rest of the top and bottom rows and of the left
# and right columns. Array.ring holds, per part, the packed FP64 bits of the one value the whole part is
# known to hold, or None when unknown; it is None for grids without an interior (fewer than 3 rows or
# columns), which are not tracked.
_ZERO_BITS = struct.pack("<d", 0.0)


def _ring_parts(H: int, W: int) -> tuple:
    return ((0, 1, 0, 1), (0, 1, W - 1, W), (H - 1, H, 0, 1), (H - 1, H, W - 1, W),
            (0, 1, 1, W - 1), (H - 1, H, 1, W - 1), (1, H - 1, 0, 1), (1, H - 1, W - 1, W))


_REGION_CACHES: dict = {}


def _region_cache(shape: tuple) -> dict:
    """Normalised slice pairs of arrays of one shape (shared by every array of that shape)."""
    c = _REGION_CACHES.get(shape)
    if c is None:
        if len(_REGION_CACHES) > 256:
            _REGION_CACHES.clear()
        c = _REGION_CACHES[shape] = {}
    return c


class Array:
    """A lazily computed FP64 grid owned by a Context."""

    def __init__(self, ctx: "Context", shape):
        self.ctx = ctx
        self.shape = (int(shape[0]), int(shape[1]))
        self.uid = next(_uids)
        self.data = ctx.backend.alloc(self.shape)  # zeros
        H, W = self.shape
        self.ring = (_ZERO_BITS,) * 8 if H >= 3 and W >= 3 else None
        self._regions = _region_cache(self.shape)

    def _region(self, key) -> tuple:
        if not isinstance(key, tuple) or len(key) != 2:
            raise IndexError("two indices or slices are required")
        a, b = key
        if type(a) is slice and type(b) is slice:
            # programs repeat the same few slices: remember their normalised form per array shape
            ck = (a.start, a.stop, a.step, b.start, b.stop, b.step)
            reg = self._regions.get(ck)
            if reg is None:
                reg = _norm(a, self.shape[0]) + _norm(b, self.shape[1])
                if len(self._regions) < 4096:
                    self._regions[ck] = reg
            return reg
        r0, r1 = _norm(a, self.shape[0])
        c0, c1 = _norm(b, self.shape[1])
        return (r0, r1, c0, c1)

    def __getitem__(self, key) -> Ref:
        return Ref(self, self._region(key))

    def __setitem__(self, key, value) -> None:
        self.ctx._assign(self, self._region(key), _wrap(value))

    def tensor(self):
        """The array's data after everything queued so far has run (syncs the context). The caller may
        write to it, so the frontend forgets what it knew of the array's ring. Later operations may move
        the array to another buffer (Jacobi chains exchange the buffers of their two arrays): call tensor()
        again to see their results."""
        self.ctx.sync()
        self.ctx.invalidate(self)
        return self.data


@dataclass(slots=True)
class Node:
    out: Array
    region: tuple
    expr: Expr
    ins: list
    ast: str
    deps: set = field(default_factory=set)  # indices of earlier nodes in the same DAG
    depth: int = 1
    chain_ok: bool = False  # whole interior, read from one array with the same known ring as `out`


class Context:
    """Records slice assignments into a DAG and runs it on the backend."""

    def __init__(self, max_depth: int = 64, backend=None, fuse: bool = True):
        if max_depth < 1:
            raise ValueError("max_depth must be >= 1")
        self.max_depth = max_depth
        self.fuse = fuse
        self.backend = backend if backend is not None else GpuBackend()
        self.nodes: list[Node] = []
        self.asts: dict[str, int] = {}
        self.stats = {"nodes": 0, "flushes": 0, "launch_groups": 0, "fused_nodes": 0, "chained_nodes": 0,
                      "chains_last_only": 0}
        # per array (uid), in the current DAG: the last node that wrote it, and the nodes that read it
        # since. Earlier writers and readers are reached through these (a later write of an array depends
        # on its earlier writers and readers), so depths and the fusion test (within runs of consecutive
        # nodes) are the same as with every per-array edge, at a cost per node that does not grow with
        # the DAG.
        self._writers: dict[int, int] = {}
        self._readers: dict[int, list] = {}

    def create_array(self, shape) -> Array:
        return Array(self, shape)

    # -- recording ----------------------------------------------------------
    def _assign(self, out: Array, region: tuple, expr: Expr) -> None:
        shape = (region[1] - region[0], region[3] - region[2])
        refs: list = []
        ast = _walk(expr, {}, refs)
        ins = []
        for r in refs:
            rr = r.region
            if (rr[1] - rr[0], rr[3] - rr[2]) != shape:
                raise ValueError(f"slice of shape {shape} assigned from a slice of another shape "
                                 "(broadcasting is not supported)")
            a = r.array
            if a is out:
                raise InPlaceDependencyError("the right side reads the array being assigned; use a second array")
            if a.ctx is not self:
                raise ValueError("arrays of different contexts")
            ins.append(a)
        self.asts[ast] = self.asts.get(ast, 0) + 1
        node = Node(out, region, expr, ins, ast)
        H, W = out.shape
        # cheap precondition of a chain here (whole interior, one other array with the same known ring);
        # the Jacobi pattern itself is matched at flush time
        node.chain_ok = out.ring is not None and region == (1, H - 1, 1, W - 1) and len(ins) > 0 and \
            ins.count(ins[0]) == len(ins) and ins[0].ring == out.ring and None not in out.ring
        self._update_ring(out, region, expr)
        in_uids = {a.uid for a in ins}
        for u in in_uids:                                       # true dependences (read after write)
            if u in self._writers:
                node.deps.add(self._writers[u])
        node.deps.update(self._readers.get(out.uid, ()))       # anti dependences (write after read)
        if out.uid in self._writers:                            # output dependences (write after write)
            node.deps.add(self._writers[out.uid])
        node.depth = 1 + max((self.nodes[k].depth for k in node.deps), default=0)
        if node.depth > self.max_depth:
            self.flush(pending=node)
            node.deps = set()
            node.depth = 1
        k = len(self.nodes)
        self.nodes.append(node)
        for u in in_uids:
            self._readers.setdefault(u, []).append(k)
        self._writers[out.uid] = k
        self._readers[out.uid] = []
        self.stats["nodes"] += 1

    def depth(self) -> int:
        return max((n.depth for n in self.nodes), default=0)

    # -- boundary rings -----------------------------------------------------
    @staticmethod
    def _update_ring(out: Array, region: tuple, expr: Expr) -> None:
        """A write to `region` of `out`: a fill covering a ring part sets it; any other touch forgets it."""
        if out.ring is None:
            return
        r0, r1, c0, c1 = region
        if r0 >= r1 or c0 >= c1:
            return
        H, W = out.shape
        if r0 >= 1 and c0 >= 1 and r1 <= H - 1 and c1 <= W - 1:  # inside the interior: no ring part
            return
        value = struct.pack("<d", float(expr.value)) if isinstance(expr, Const) else None
        ring = list(out.ring)
        for k, (a0, a1, b0, b1) in enumerate(_ring_parts(*out.shape)):
            if r1 <= a0 or a1 <= r0 or c1 <= b0 or b1 <= c0:
                continue
            covers = r0 <= a0 and a1 <= r1 and c0 <= b0 and b1 <= c1
            ring[k] = value if covers else None
        out.ring = tuple(ring)

    def invalidate(self, array: Array) -> None:
        """Forget what is known of `array`'s ring (call after writing its data outside the frontend)."""
        if array.ring is not None:
            array.ring = (None,) * 8

    def _chain_at(self, groups: list, i: int) -> list:
        """Node indices of the Jacobi chain that starts at group i (at least 2 nodes), else []."""
        chain = []
        prev = None
        for g in groups[i:]:
            if len(g) != 1:
                break
            n = self.nodes[g[0]]
            if not n.chain_ok:
                break
            jac = match_jacobi(n)
            if jac is None or jac[0].shape != n.out.shape:
                break
            src, c = jac
            if prev is not None:
                psrc, pout, pc = prev
                if src is not pout or n.out is not psrc or struct.pack("<d", c) != struct.pack("<d", pc):
                    break
            chain.append(g[0])
            prev = (src, n.out, c)
        return chain if len(chain) >= 2 else []

    # -- execution ----------------------------------------------------------
    def _groups(self) -> list[list[int]]:
        """Fusion: runs of consecutive nodes with the same output shape and no path between them."""
        groups: list[list[int]] = []
        for k, n in enumerate(self.nodes):
            if self.fuse and groups:
                g = groups[-1]
                first = self.nodes[g[0]]
                same_shape = (first.region[1] - first.region[0], first.region[3] - first.region[2]) == \
                    (n.region[1] - n.region[0], n.region[3] - n.region[2])
                independent = not any(j in n.deps for j in g)
                if same_shape and independent and self.backend.fusable(first, n):
                    g.append(k)
                    continue
            groups.append([k])
        return groups

    def flush(self, pending: Node | None = None) -> None:
        """Send the current DAG to the backend (program order is a topological order). `pending` is the
        node whose recording caused the flush (it runs in the next DAG): when it overwrites the whole
        interior of the array a final Jacobi chain leaves iterate m-1 in, that iterate is dead and the
        chain need not produce it."""
        if not self.nodes:
            return
        groups = self._groups()
        i = 0
        while i < len(groups):
            chain = self._chain_at(groups, i) if hasattr(self.backend, "run_chain") else []
            if chain:
                nodes = [self.nodes[k] for k in chain]
                last = nodes[-1]
                prev = match_jacobi(last)[0]  # the array holding iterate m-1 afterwards
                H, W = prev.shape
                dead = pending is not None and i + len(chain) == len(groups) and pending.out is prev and \
                    pending.region == (1, H - 1, 1, W - 1)
                if dead:
                    self.backend.run_chain(nodes, keep_previous=False)
                    self.stats["chains_last_only"] += 1
                else:
                    self.backend.run_chain(nodes)
                self.stats["launch_groups"] += 1
                self.stats["chained_nodes"] += len(chain)
                i += len(chain)
                continue
            g = groups[i]
            self.backend.run([self.nodes[k] for k in g])
            self.stats["launch_groups"] += 1
            if len(g) > 1:
                self.stats["fused_nodes"] += len(g)
            i += 1
        self.nodes = []
        self._writers.clear()
        self._readers.clear()
        self.stats["flushes"] += 1

    def sync(self) -> None:
        self.flush()
        self.backend.synchronize()

    def distinct_asts(self) -> int:
        return len(self.asts)


# ---------------------------------------------------------------------------
# Pattern recognition shared by backends
# ---------------------------------------------------------------------------

def _flatten_sum(e: Expr) -> list:
    """Left-associated '+' chain -> list of terms, in order."""
    terms = []
    while isinstance(e, BinOp) and e.op == "+":
        terms.append(e.b)
        e = e.a
    terms.append(e)
    return terms[::-1]


_JACOBI_MATCH: dict = {}
_MISSING = object()


def match_jacobi(node: Node):
    """c * (((N + S) + W) + E) on the output region -> (array, c) or None. The parameterised AST text
    (structure, constants, which array each reference names and its region) and the output region
    decide the match, so the answer is remembered per (AST, region)."""
    key = (node.ast, node.region)
    c = _JACOBI_MATCH.get(key, _MISSING)
    if c is _MISSING:
        m = _match_jacobi_tree(node)
        c = None if m is None else m[1]
        if len(_JACOBI_MATCH) > 65536:
            _JACOBI_MATCH.clear()
        _JACOBI_MATCH[key] = c
    return None if c is None else (node.ins[0], c)


def _match_jacobi_tree(node: Node):
    e = node.expr
    if not (isinstance(e, BinOp) and e.op == "*" and isinstance(e.a, Const)):
        return None
    terms = _flatten_sum(e.b)
    if len(terms) != 4 or not all(isinstance(t, Ref) for t in terms):
        return None
    src = terms[0].array
    if any(t.array is not src for t in terms):
        return None
    r0, r1, c0, c1 = node.region
    want = [(r0 - 1, r1 - 1, c0, c1), (r0 + 1, r1 + 1, c0, c1), (r0, r1, c0 - 1, c1 - 1), (r0, r1, c0 + 1, c1 + 1)]
    if [t.region for t in terms] != want:
        return None
    return src, e.a.value


def match_star(node: Node):
    """c0*A + cN1*A[up] + cS1*A[down] + cW1*A[left] + cE1*A[right] + ... -> (array, spec) or None."""
    terms = _flatten_sum(node.expr)
    if (len(terms) - 1) % 4 != 0 or len(terms) < 5:
        return None
    R = (len(terms) - 1) // 4
    coefs, refs = [], []
    for t in terms:
        if isinstance(t, BinOp) and t.op == "*" and isinstance(t.a, Const) and isinstance(t.b, Ref):
            coefs.append(t.a.value)
            refs.append(t.b)
        else:
            return None
    src = refs[0].array
    if any(r.array is not src for r in refs):
        return None
    H, W = node.out.shape
    if src.shape != node.out.shape or node.region != (R, H - R, R, W - R):
        return None
    r0, r1, c0, c1 = node.region
    want = [(r0, r1, c0, c1)]
    for k in range(1, R + 1):
        want += [(r0 - k, r1 - k, c0, c1), (r0 + k, r1 + k, c0, c1), (r0, r1, c0 - k, c1 - k), (r0, r1, c0 + k, c1 + k)]
    if [r.region for r in refs] != want:
        return None
    c0_ = coefs[0]
    cn = coefs[1::4]
    cs = coefs[2::4]
    cw = coefs[3::4]
    ce = coefs[4::4]
    return src, (c0_, cn, cs, cw, ce)


# ---------------------------------------------------------------------------
# Expression programs for generated kernels
# ---------------------------------------------------------------------------

EXPR_MAX_IN = 16   # input slots of one generated kernel (libsten limit)
EXPR_MAX_OUT = 8   # outputs of one generated kernel (libsten limit)


def node_kind(node: Node) -> str:
    """'fill', 'jacobi', 'star' (hand-written kernels) or 'expr' (generated kernel)."""
    if isinstance(node.expr, Const):
        return "fill"
    if match_jacobi(node) is not None and node.ins[0].shape == node.out.shape:
        return "jacobi"
    if match_star(node) is not None:
        return "star"
    return "expr"


def build_program(nodes: list) -> tuple:
    """One postfix program for a fused group of same-shape nodes (grammar in include/sten.h).

    Returns (text, ins, outs, rows, cols): ins and outs are (array, r0, c0) triples, the element of
    each array aligned with output point (0, 0). An input slot is one array seen from one output
    origin; every load is an offset from it. Constants are written as exact hexadecimal floats.
    """
    r0, r1, c0, c1 = nodes[0].region
    rows, cols = r1 - r0, c1 - c0
    slots: dict = {}
    ins: list = []
    outs: list = []
    texts = []
    for n in nodes:
        o0, o1, p0, p1 = n.region
        if (o1 - o0, p1 - p0) != (rows, cols):
            raise ValueError("fused nodes must have one output shape")
        toks: list = []

        def emit(e):
            if isinstance(e, Const):
                toks.append("C" + float(e.value).hex())
            elif isinstance(e, Ref):
                key = (e.array.uid, o0, p0)
                if key not in slots:
                    slots[key] = len(ins)
                    ins.append((e.array, o0, p0))
                toks.append(f"L{slots[key]},{e.region[0] - o0},{e.region[2] - p0}")
            elif isinstance(e, Unary):
                emit(e.a)
                toks.append({"neg": "N", "sq": "Q"}[e.op])
            else:
                emit(e.a)
                emit(e.b)
                toks.append(e.op)

        emit(n.expr)
        texts.append(" ".join(toks))
        outs.append((n.out, o0, p0))
    return "; ".join(texts), ins, outs, rows, cols


def split_for_limits(nodes: list) -> list:
    """A fused group as consecutive chunks that each fit one generated kernel's slot and output limits;
    returns build_program's result for each chunk."""
    progs = []
    cur: list = []
    prog = None
    for n in nodes:
        trial = build_program(cur + [n])
        if cur and (len(trial[1]) > EXPR_MAX_IN or len(trial[2]) > EXPR_MAX_OUT):
            progs.append(prog)
            cur, trial = [n], build_program([n])
        else:
            cur = cur + [n]
        prog = trial
    if prog is not None:
        progs.append(prog)
    for p in progs:
        if len(p[1]) > EXPR_MAX_IN:
            raise NotImplementedError(f"an expression reads more than {EXPR_MAX_IN} slices of distinct arrays")
    return progs


def swap_chain_buffers(chain: list, lands_in_b: bool) -> None:
    """After a chain that produced only its last iterate: if the iterate landed in the buffer of the array
    that one node at a time would have left iterate m-1 in, the two arrays exchange buffers, so that the
    chain's last node's output array holds it. Both arrays carry the same ring (a chain's precondition)
    and the other one's interior is dead, so nothing a program can read changes; only a buffer handed out
    earlier by tensor() no longer belongs to the same array (tensor() is to be called again after more
    operations)."""
    a = match_jacobi(chain[0])[0]
    b = chain[0].out
    m = len(chain)
    if lands_in_b != bool(m % 2):
        a.data, b.data = b.data, a.data


# ---------------------------------------------------------------------------
# GPU backend (libsten)
# ---------------------------------------------------------------------------

class GpuBackend:
    """Runs DAG nodes with libsten kernels on the current HIP stream."""

    def __init__(self, device=None):
        import torch

        from . import ops

        self.torch = torch
        self.ops = ops
        self.device = device or torch.device("cuda")
        self._programs: dict = {}

    def alloc(self, shape):
        return self.torch.zeros(shape, dtype=self.torch.float64, device=self.device)

    def fusable(self, a: Node, b: Node) -> bool:
        ka, kb = node_kind(a), node_kind(b)
        if ka == "star" and kb == "star":
            sa, sb = match_star(a), match_star(b)
            return sa[0] is sb[0] and len(sa[1][1]) == len(sb[1][1])
        return ka == "expr" and kb == "expr"

    def run(self, group: list) -> None:
        from . import _lib
        from .ops import _ld, _stream_ptr

        kind = node_kind(group[0])
        if len(group) > 1 and kind == "star":  # fused star stencils reading one array
            src = match_star(group[0])[0]
            specs = [match_star(n)[1] for n in group]
            self.ops.star(src.data, specs, outs=[n.out.data for n in group])
            return
        if len(group) == 1 and kind != "expr":
            n = group[0]
            H, W = n.out.shape
            r0, r1, c0, c1 = n.region
            if kind == "fill":
                _lib.call("sten_fill_rect_f64", n.out.data.data_ptr(), H, W, _ld(n.out.data), r0, r1, c0, c1,
                          float(n.expr.value), _stream_ptr())
                return
            if kind == "jacobi":
                src, c = match_jacobi(n)
                # view of the region grown by one: the sweep writes exactly its interior
                vs = src.data[r0 - 1:r1 + 1, c0 - 1:c1 + 1]
                vd = n.out.data[r0 - 1:r1 + 1, c0 - 1:c1 + 1]
                _lib.call("sten_sweep_f64", vs.data_ptr(), vd.data_ptr(), vs.shape[0], vs.shape[1],
                          _ld(src.data), float(c), _stream_ptr())
                return
            s = match_star(n)
            self.ops.star(s[0].data, [s[1]], outs=[n.out.data])
            return
        # programs depend only on the nodes' ASTs, regions and arrays: cache them (iterations that
        # swap arrays alternate between a few keys)
        key = tuple((n.ast, n.region, tuple(a.uid for a in n.ins), n.out.uid) for n in group)
        progs = self._programs.get(key)
        if progs is None:
            progs = split_for_limits(group)
            if len(self._programs) > 4096:
                self._programs.clear()
            self._programs[key] = progs
        for text, ins, outs, rows, cols in progs:
            self.ops.expr_run(text, [(a.data, r0, c0) for a, r0, c0 in ins],
                              [(a.data, r0, c0) for a, r0, c0 in outs], rows, cols)

    def run_chain(self, chain: list, keep_previous: bool = True) -> None:
        """Jacobi nodes ping-ponging between two arrays with equal rings: one libsten chain call. Without
        keep_previous only the last iterate is produced, by the fewest blocked launches; when those leave it
        in the other array, the two arrays exchange buffers (swap_chain_buffers)."""
        from . import _lib
        from .ops import _ld, _stream_ptr

        a, c = match_jacobi(chain[0])
        b = chain[0].out
        H, W = b.shape
        if a.data.stride() != b.data.stride():
            for n in chain:
                self.run([n])
            return
        if keep_previous:
            _lib.call("sten_sweep_chain_f64", a.data.data_ptr(), b.data.data_ptr(), H, W, _ld(a.data), len(chain),
                      float(c), _stream_ptr())
            return
        lands_in_b = ctypes.c_int32(0)
        _lib.call("sten_sweep_chain_last_f64", a.data.data_ptr(), b.data.data_ptr(), H, W, _ld(a.data), len(chain),
                  float(c), ctypes.byref(lands_in_b), _stream_ptr())
        swap_chain_buffers(chain, bool(lands_in_b.value))

    def synchronize(self) -> None:
        self.torch.cuda.synchronize()
