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
  tree (AST) over slices of other arrays, scalars, +, - and *; the tree is
  parameterised (arrays are placeholders), so iterations that only swap arrays
  share one AST;
* an assignment whose right side reads the array it writes is rejected
  (``InPlaceDependencyError``), which is why the listing uses two arrays;
* nodes form a DAG with true, anti and output dependencies tracked per array
  (conservative: per array, not per index);
* the DAG is sent to the backend when ``sync()`` is called or when its depth
  would exceed ``max_depth``; kernel launches are asynchronous, so the Python
  side keeps building the next DAG while the GPU executes the previous one
  (pipelining);
* before execution, consecutive nodes with the same output region and no path
  between them are fused (node fusion).

Backend (no run-time code generation): recognised ASTs map to libsten kernels -
scalar fills -> ``sten_fill_rect_f64``; the listing's update
``c*(N + S + W + E)`` on any rectangle -> ``sten_sweep_f64`` on a view; a
left-to-right sum of ``coef * shifted slice`` terms in the canonical star
order -> ``sten_star_f64`` (fused nodes that read the same array share one
launch). Other expressions raise ``NotImplementedError``.
"""

from __future__ import annotations

import itertools
from dataclasses import dataclass, field

__all__ = ["Context", "Array", "InPlaceDependencyError"]


class InPlaceDependencyError(ValueError):
    """The right side of an assignment reads the array being assigned."""


# ---------------------------------------------------------------------------
# Expressions
# ---------------------------------------------------------------------------

class Expr:
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


@dataclass(eq=False)
class Const(Expr):
    value: float


@dataclass(eq=False)
class Ref(Expr):
    array: "Array"
    region: tuple  # (r0, r1, c0, c1), half-open, step 1


@dataclass(eq=False)
class BinOp(Expr):
    op: str
    a: Expr
    b: Expr


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


def _arrays(e: Expr, acc: list) -> list:
    if isinstance(e, Ref):
        acc.append(e.array)
    elif isinstance(e, BinOp):
        _arrays(e.a, acc)
        _arrays(e.b, acc)
    return acc


def _structure(e: Expr, names: dict) -> str:
    """Parameterised AST text: arrays become placeholders in order of first use."""
    if isinstance(e, Const):
        return repr(e.value)
    if isinstance(e, Ref):
        k = names.setdefault(e.array.uid, f"A{len(names)}")
        return f"{k}[{e.region}]"
    return f"({_structure(e.a, names)}{e.op}{_structure(e.b, names)})"


# ---------------------------------------------------------------------------
# Arrays and DAG nodes
# ---------------------------------------------------------------------------

_uids = itertools.count()


class Array:
    """A lazily computed FP64 grid owned by a Context."""

    def __init__(self, ctx: "Context", shape):
        self.ctx = ctx
        self.shape = (int(shape[0]), int(shape[1]))
        self.uid = next(_uids)
        self.data = ctx.backend.alloc(self.shape)

    def _region(self, key) -> tuple:
        if not isinstance(key, tuple) or len(key) != 2:
            raise IndexError("two indices or slices are required")
        r0, r1 = _norm(key[0], self.shape[0])
        c0, c1 = _norm(key[1], self.shape[1])
        return (r0, r1, c0, c1)

    def __getitem__(self, key) -> Ref:
        return Ref(self, self._region(key))

    def __setitem__(self, key, value) -> None:
        self.ctx._assign(self, self._region(key), _wrap(value))

    def tensor(self):
        """The array's data after everything queued so far has run (syncs the context)."""
        self.ctx.sync()
        return self.data


@dataclass
class Node:
    out: Array
    region: tuple
    expr: Expr
    ins: list
    ast: str
    deps: set = field(default_factory=set)  # indices of earlier nodes in the same DAG
    depth: int = 1


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
        self.stats = {"nodes": 0, "flushes": 0, "launch_groups": 0, "fused_nodes": 0}

    def create_array(self, shape) -> Array:
        return Array(self, shape)

    # -- recording ----------------------------------------------------------
    def _assign(self, out: Array, region: tuple, expr: Expr) -> None:
        ins = _arrays(expr, [])
        if any(a is out for a in ins):
            raise InPlaceDependencyError("the right side reads the array being assigned; use a second array")
        for a in ins:
            if a.ctx is not self:
                raise ValueError("arrays of different contexts")
        ast = _structure(expr, {})
        self.asts[ast] = self.asts.get(ast, 0) + 1
        node = Node(out, region, expr, ins, ast)
        for k, m in enumerate(self.nodes):
            true_dep = any(a is m.out for a in ins)
            anti_dep = any(a is out for a in m.ins)
            out_dep = m.out is out
            if true_dep or anti_dep or out_dep:
                node.deps.add(k)
        node.depth = 1 + max((self.nodes[k].depth for k in node.deps), default=0)
        if node.depth > self.max_depth:
            self.flush()
            node.deps = set()
            node.depth = 1
        self.nodes.append(node)
        self.stats["nodes"] += 1

    def depth(self) -> int:
        return max((n.depth for n in self.nodes), default=0)

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

    def flush(self) -> None:
        """Send the current DAG to the backend (program order is a topological order)."""
        if not self.nodes:
            return
        groups = self._groups()
        for g in groups:
            self.backend.run([self.nodes[k] for k in g])
            self.stats["launch_groups"] += 1
            if len(g) > 1:
                self.stats["fused_nodes"] += len(g)
        self.nodes = []
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


def match_jacobi(node: Node):
    """c * (((N + S) + W) + E) on the output region -> (array, c) or None."""
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

    def alloc(self, shape):
        return self.torch.zeros(shape, dtype=self.torch.float64, device=self.device)

    def fusable(self, a: Node, b: Node) -> bool:
        sa, sb = match_star(a), match_star(b)
        return sa is not None and sb is not None and sa[0] is sb[0] and len(sa[1][1]) == len(sb[1][1])

    def run(self, group: list) -> None:
        from . import _lib
        from .ops import _ld, _stream_ptr

        if len(group) > 1:  # fused star stencils reading one array
            src = match_star(group[0])[0]
            specs = [match_star(n)[1] for n in group]
            self.ops.star(src.data, specs, outs=[n.out.data for n in group])
            return
        n = group[0]
        H, W = n.out.shape
        r0, r1, c0, c1 = n.region
        if isinstance(n.expr, Const):
            _lib.call("sten_fill_rect_f64", n.out.data.data_ptr(), H, W, _ld(n.out.data), r0, r1, c0, c1,
                      float(n.expr.value), _stream_ptr())
            return
        m = match_jacobi(n)
        if m is not None:
            src, c = m
            if src.shape != n.out.shape:
                raise NotImplementedError("sweep between arrays of different shapes")
            # view of the region grown by one: the sweep writes exactly its interior
            vs = src.data[r0 - 1:r1 + 1, c0 - 1:c1 + 1]
            vd = n.out.data[r0 - 1:r1 + 1, c0 - 1:c1 + 1]
            _lib.call("sten_sweep_f64", vs.data_ptr(), vd.data_ptr(), vs.shape[0], vs.shape[1], _ld(src.data),
                      float(c), _stream_ptr())
            return
        s = match_star(n)
        if s is not None:
            self.ops.star(s[0].data, [s[1]], outs=[n.out.data])
            return
        raise NotImplementedError(f"expression not supported by the backend: {n.ast}")

    def synchronize(self) -> None:
        self.torch.cuda.synchronize()
