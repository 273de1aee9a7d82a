"""A frontend backend that runs every DAG node eagerly with plain NumPy (CPU, test infrastructure).

It evaluates each node's expression tree element-wise in FP64, operation by
operation in tree order, exactly as NumPy evaluates the same slice expression,
and records the launch groups the frontend formed. Fusion follows the GPU
backend's rules (generated-kernel nodes fuse with each other, star stencils of
one array fuse), so group structure can be checked on the CPU.
"""

import numpy as np

import oracle
from paper_2512_19851_amd import frontend as fe


class NumpyBackend:
    def __init__(self, chain_levels: int = 10):
        self.groups = []
        self.chains = []
        self.swaps = 0
        self.chain_levels = chain_levels

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

    def run_chain(self, chain, keep_previous=True):
        """A model of the library's chain plans on the CPU. Both iterates kept: the first m-1 sweeps as k
        blocked passes (each pass is `lev` sweeps of the oracle from the pass's source, that array's ring at
        every level), k chosen with the parity that ends in the array of iterate m-1, then one plain sweep.
        Last iterate only: all m sweeps as the fewest passes, the arrays exchanging buffers when those end
        in the other array (as the GPU backend does), and the dead array's interior then poisoned with NaN,
        so that a result that depended on it would show."""
        a, c = fe.match_jacobi(chain[0])
        b = chain[0].out
        m = len(chain)
        self.chains.append(m if keep_previous else -m)
        L = self.chain_levels
        n = m - 1 if keep_previous else m
        src = a
        if L > 1 and n >= 2:
            k = -(-n // L)
            if keep_previous and k % 2 != n % 2:
                k += 1
            base, extra = divmod(n, k)
            for j in range(1, k + 1):
                dst = b if j % 2 else a
                lev = base + (1 if j <= extra else 0)
                dst.data[1:-1, 1:-1] = oracle.jacobi5(src.data, lev, c)[1:-1, 1:-1]
                src = dst
        else:
            for j in range(1, n + 1):
                dst = b if j % 2 else a
                dst.data[1:-1, 1:-1] = oracle.jacobi5(src.data, 1, c)[1:-1, 1:-1]
                src = dst
        if keep_previous:
            other = b if src is a else a
            other.data[1:-1, 1:-1] = oracle.jacobi5(src.data, 1, c)[1:-1, 1:-1]
            return
        fe.swap_chain_buffers(chain, src is b)
        self.swaps += int((src is b) != bool(m % 2))
        dead = a if m % 2 else b  # the array one node at a time would leave iterate m-1 in
        dead.data[1:-1, 1:-1] = np.nan

    def synchronize(self):
        pass
