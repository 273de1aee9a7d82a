"""A frontend backend that runs every DAG node eagerly with plain NumPy (CPU, test infrastructure).

It evaluates each node's expression tree element-wise in FP64, operation by
operation in tree order, exactly as NumPy evaluates the same slice expression,
and records the launch groups the frontend formed. Fusion follows the GPU
backend's rules (generated-kernel nodes fuse with each other, star stencils of
one array fuse), so group structure can be checked on the CPU.
"""

import numpy as np

from paper_2512_19851_amd import frontend as fe


class NumpyBackend:
    def __init__(self):
        self.groups = []

    def alloc(self, shape):
        return np.zeros(shape)

    def fusable(self, a, b):
        ka, kb = fe.node_kind(a), fe.node_kind(b)
        if ka == "star" and kb == "star":
            sa, sb = fe.match_star(a), fe.match_star(b)
            return sa[0] is sb[0] and len(sa[1][1]) == len(sb[1][1])
        return ka == "expr" and kb == "expr"

    def _eval(self, e):
        if isinstance(e, fe.Const):
            return e.value
        if isinstance(e, fe.Ref):
            r0, r1, c0, c1 = e.region
            return e.array.data[r0:r1, c0:c1].copy()
        if isinstance(e, fe.Unary):
            a = self._eval(e.a)
            return -a if e.op == "neg" else a * a
        a, b = self._eval(e.a), self._eval(e.b)
        return {"+": lambda: a + b, "-": lambda: a - b, "*": lambda: a * b, "/": lambda: a / b}[e.op]()

    def run(self, group):
        self.groups.append([(n.ast, fe.match_jacobi(n) is not None, fe.match_star(n) is not None) for n in group])
        vals = [self._eval(n.expr) for n in group]  # fused nodes read before any writes
        for n, v in zip(group, vals):
            r0, r1, c0, c1 = n.region
            n.out.data[r0:r1, c0:c1] = v

    def synchronize(self):
        pass
