"""CPU simulator of the schedules printed by ffp_plan_describe.

Test infrastructure: it executes, in program order, the block operations of
one fsyrk_modp schedule on numpy views of three byte buffers (the operand A,
the output C and the workspace), each operation written from its definition
in Algorithm 2 of the paper (pre-additions with the skew-orthogonal Y,
products, post-additions) and from the placements of Tables 3 and 4.  numpy
refuses a view that leaves its buffer, so the simulation is also a bounds
check of every view the schedule uses.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

CLS_F64, CLS_I8, CLS_LIMB2, CLS_LIMB3 = 0, 1, 2, 3
(OP_S1S2, OP_S34, OP_GEMM, OP_SYRK, OP_POSTADD, OP_ADDLOW, OP_SAVEC22, OP_MIRROR, OP_PACK, OP_COPY,
 OP_LINCOMB, OP_LCT) = range(12)


@dataclass
class View:
    buf: int
    off: int
    ld: int
    plane: int


@dataclass
class Op:
    kind: int
    cls: int
    src_cls: int
    mode: int
    m: int
    n: int
    k: int
    m_src: int
    k_src: int
    alpha: int
    beta: int
    level: int
    v: list = field(default_factory=list)
    coef: list = field(default_factory=lambda: [1] * 5)


@dataclass
class Plan:
    cls: int
    depth: int
    n_pad: int
    k_pad: int
    ws: int
    ya: int
    yb: int
    ops: list


def parse(text: str) -> Plan:
    lines = [ln for ln in text.strip().splitlines() if ln.strip()]
    head = dict(kv.split("=") for kv in lines[0].split()[1:])
    ops = []
    for ln in lines[1:]:
        f = [int(x) for x in ln.split()[1:]]
        views = [View(*f[12 + 4 * i: 16 + 4 * i]) for i in range(6)]
        coef = f[36:41] if len(f) >= 41 else [1] * 5
        ops.append(Op(*f[:12], v=views, coef=coef))
    return Plan(int(head["cls"]), int(head["depth"]), int(head["n_pad"]), int(head["k_pad"]),
                int(head["ws"]), int(head["ya"]), int(head["yb"]), ops)


def matmul_nt(X, Y):
    """Exact X Y^T of non-negative residues: int64 while every sum stays
    below 2^63, Python integers otherwise (large p)."""
    big = int(max(X.max(initial=0), Y.max(initial=0)))
    if big * big * max(X.shape[1], 1) < 2**62:
        return X.astype(np.int64) @ Y.astype(np.int64).T
    if X.size == 0 or Y.size == 0:
        return np.zeros((X.shape[0], Y.shape[0]), dtype=np.int64)
    return X.astype(object) @ Y.astype(object).T


class Sim:
    def __init__(self, bufs, p: int, plan: Plan):
        self.bufs = bufs
        self.p = p
        self.plan = plan

    # ---- storage access -------------------------------------------------
    def _nd(self, v: View, dtype, rows, cols, extra=0):
        es = np.dtype(dtype).itemsize
        return np.ndarray((rows, cols), dtype=dtype, buffer=self.bufs[v.buf],
                          offset=v.off + extra * es, strides=(v.ld * es, es))

    def get(self, v: View, cls: int, rows: int, cols: int) -> np.ndarray:
        p = self.p
        if rows == 0 or cols == 0:
            return np.zeros((rows, cols), dtype=np.int64)
        if cls == CLS_F64:
            return self._nd(v, np.uint32, rows, cols).astype(np.int64)
        if cls == CLS_I8:
            return self._nd(v, np.int8, rows, cols).astype(np.int64) % p
        if cls == CLS_LIMB3:   # planes lo, mid, hi
            lo = self._nd(v, np.int8, rows, cols).astype(np.int64)
            mid = self._nd(v, np.int8, rows, cols, extra=v.plane).astype(np.int64)
            hi = self._nd(v, np.int8, rows, cols, extra=2 * v.plane).astype(np.int64)
            return (lo + 256 * mid + 65536 * hi) % p
        hi = self._nd(v, np.int8, rows, cols).astype(np.int64)
        lo = self._nd(v, np.int8, rows, cols, extra=v.plane).astype(np.int64)
        return (256 * hi + lo) % p

    def put(self, v: View, cls: int, vals: np.ndarray):
        p = self.p
        rows, cols = vals.shape
        if rows == 0 or cols == 0:
            return
        vals = np.asarray(vals, dtype=np.int64) % p
        if cls == CLS_F64:
            self._nd(v, np.uint32, rows, cols)[...] = vals.astype(np.uint32)
        elif cls == CLS_I8:
            x = np.where(vals > (p - 1) // 2, vals - p, vals)
            assert np.all(np.abs(x) <= 127)
            self._nd(v, np.int8, rows, cols)[...] = x.astype(np.int8)
        elif cls == CLS_LIMB3:
            x = np.where(vals > (p - 1) // 2, vals - p, vals)
            lo = ((x + 128) & 255) - 128
            y = (x - lo) >> 8
            mid = ((y + 128) & 255) - 128
            hi = (y - mid) >> 8
            assert np.all((hi >= -128) & (hi <= 127))
            self._nd(v, np.int8, rows, cols)[...] = lo.astype(np.int8)
            self._nd(v, np.int8, rows, cols, extra=v.plane)[...] = mid.astype(np.int8)
            self._nd(v, np.int8, rows, cols, extra=2 * v.plane)[...] = hi.astype(np.int8)
        else:
            x = np.where(vals <= 32639, vals, vals - p)
            lo = ((x + 128) & 255) - 128
            hi = (x - lo) >> 8
            assert np.all((hi >= -128) & (hi <= 127))
            self._nd(v, np.int8, rows, cols)[...] = hi.astype(np.int8)
            self._nd(v, np.int8, rows, cols, extra=v.plane)[...] = lo.astype(np.int8)

    # ---- operations ---------------------------------------------------------
    def times_y(self, X):
        """X Y with Y = [[a I, b I], [-b I, a I]] (b = 0: Y = a I)."""
        a, b, p = self.plan.ya, self.plan.yb, self.p
        if b == 0:
            return (a * X) % p
        h2 = X.shape[1] // 2
        L, R = X[:, :h2], X[:, h2:]
        return np.concatenate([(a * L - b * R) % p, (b * L + a * R) % p], axis=1)

    def run(self, order=None):
        ops = self.plan.ops if order is None else [self.plan.ops[i] for i in order]
        for op in ops:
            getattr(self, f"op{op.kind}")(op)

    def op0(self, o):   # S1 = (A21 - A11) Y, S2 = A22 - A21 Y
        m, h, c, p = o.m, o.k, o.cls, self.p
        A11, A21, A22 = (self.get(o.v[i], c, m, h) for i in range(3))
        S1 = self.times_y((A21 - A11) % p)
        S2 = (A22 - self.times_y(A21)) % p
        self.put(o.v[3], c, S1)
        self.put(o.v[4], c, S2)

    def op1(self, o):   # S3 = S1 - A22 ; S4 = S3 + A12
        m, h, c, p = o.m, o.k, o.cls, self.p
        if o.mode & 1:
            S3 = (self.get(o.v[0], c, m, h) - self.get(o.v[1], c, m, h)) % p
            self.put(o.v[3], c, S3)
        else:
            S3 = self.get(o.v[3], c, m, h)
        if o.mode & 2:
            self.put(o.v[4], c, (S3 + self.get(o.v[2], c, m, h)) % p)

    def op2(self, o):   # C = alpha A B^T + beta C (mode bit 0: lower triangle only)
        A = self.get(o.v[0], o.cls, o.m, o.k)
        B = self.get(o.v[1], o.cls, o.n, o.k)
        C = self.get(o.v[2], CLS_F64, o.m, o.n)
        R = (o.alpha * (matmul_nt(A, B) % self.p) + o.beta * C) % self.p
        if o.mode & 1:
            low = np.tril(np.ones((o.m, o.n), dtype=bool))
            C[low] = R[low]
            R = C
        self.put(o.v[2], CLS_F64, R)

    def op3(self, o):   # lower(C) = alpha A A^T + beta lower(C)
        n = o.m
        A = self.get(o.v[0], o.cls, n, o.k)
        C = self.get(o.v[1], CLS_F64, n, n)
        R = (o.alpha * (matmul_nt(A, A) % self.p) + o.beta * C) % self.p
        low = np.tril(np.ones((n, n), dtype=bool))
        C[low] = R[low]
        self.put(o.v[1], CLS_F64, C)

    def op4(self, o):   # U1 = P1+P5, U2 = U1+P4, U4 = U2+P3, U5 = U2+P4^T (+beta C22_in)
        m, p = o.m, self.p
        low = np.tril(np.ones((m, m), dtype=bool))
        P1 = self.get(o.v[0], CLS_F64, m, m)
        P5 = self.get(o.v[1], CLS_F64, m, m)
        P4T = self.get(o.v[2], CLS_F64, m, m)
        P3 = self.get(o.v[3], CLS_F64, m, m)
        L1 = np.where(low, (P1 + P5) % p, 0)
        U1 = L1 + np.tril(L1, -1).T
        U2 = (U1 + P4T.T) % p
        U4 = (U2 + P3) % p
        U5 = (U2 + P4T) % p
        if o.beta:
            up = self.get(o.v[4], CLS_F64, m, m)
            d = self.get(o.v[5], CLS_F64, 1, m)[0]
            C22in = np.triu(up, 1).T + np.diag(d)
            U5 = (U5 + o.beta * C22in) % p
        self.put(o.v[3], CLS_F64, U4)
        C22 = self.get(o.v[2], CLS_F64, m, m)
        C22[low] = U5[low]
        self.put(o.v[2], CLS_F64, C22)

    def op5(self, o):   # lower(Z) = lower(X) + lower(Y)
        m = o.m
        low = np.tril(np.ones((m, m), dtype=bool))
        X = self.get(o.v[0], CLS_F64, m, m)
        Y = self.get(o.v[1], CLS_F64, m, m)
        Z = self.get(o.v[2], CLS_F64, m, m)
        Z[low] = ((X + Y) % self.p)[low]
        self.put(o.v[2], CLS_F64, Z)

    def op6(self, o):   # Up(dst) = Low(src)^T strictly, dvec = diag(src)
        m = o.m
        S = self.get(o.v[0], CLS_F64, m, m)
        D = self.get(o.v[1], CLS_F64, m, m)
        up = np.triu(np.ones((m, m), dtype=bool), 1)
        D[up] = S.T[up]
        self.put(o.v[1], CLS_F64, D)
        self.put(o.v[2], CLS_F64, np.diag(S)[None, :])

    def op7(self, o):   # Up(C) = Low(C)^T (mode bit 0: -Low(C)^T)
        m = o.m
        C = self.get(o.v[0], CLS_F64, m, m)
        up = np.triu(np.ones((m, m), dtype=bool), 1)
        C[up] = (-C.T[up] % self.p) if o.mode & 1 else C.T[up]
        self.put(o.v[0], CLS_F64, C)

    def op11(self, o):  # v5 = sum coef_i op_i(v_i) mod p (bit 3 + i: transpose; bit 8: lower only)
        acc = np.zeros((o.m, o.k), dtype=object)
        for i in range(o.mode & 7):
            if (o.mode >> (3 + i)) & 1:
                X = self.get(o.v[i], CLS_F64, o.k, o.m).T
            else:
                X = self.get(o.v[i], CLS_F64, o.m, o.k)
            acc = acc + int(o.coef[i]) * X.astype(object)
        R = np.array(acc % self.p, dtype=np.int64)
        if (o.mode >> 8) & 1:
            C = self.get(o.v[5], CLS_F64, o.m, o.k)
            low = np.tril(np.ones((o.m, o.k), dtype=bool))
            C[low] = R[low]
            R = C
        self.put(o.v[5], CLS_F64, R)

    def op8(self, o):   # pack with zero padding
        src = self.get(o.v[0], o.src_cls, o.m_src, o.k_src)
        dst = np.zeros((o.m, o.k), dtype=np.int64)
        dst[: o.m_src, : o.k_src] = src
        self.put(o.v[1], o.cls, dst)

    def op10(self, o):  # v5 = sum of +-v_i mod p (bit 3 + i of mode: subtract)
        acc = np.zeros((o.m, o.k), dtype=np.int64)
        for i in range(o.mode & 7):
            X = self.get(o.v[i], CLS_F64, o.m, o.k)
            acc = acc - X if (o.mode >> (3 + i)) & 1 else acc + X
        self.put(o.v[5], CLS_F64, acc % self.p)

    def op9(self, o):   # copy
        X = self.get(o.v[0], CLS_F64, o.m, o.n)
        Y = self.get(o.v[1], CLS_F64, o.m, o.n)
        if o.mode & 1:
            low = np.tril(np.ones((o.m, o.n), dtype=bool))
            Y[low] = X[low]
        else:
            Y = X
        self.put(o.v[1], CLS_F64, Y)


def simulate_complex(plan_text: str, p: int, A: np.ndarray, order=None):
    """Run a complex schedule (A of shape (2, n, k), planes stacked) on host
    copies; returns the (2, n, n) result planes."""
    plan = parse(plan_text)
    _, n, k = A.shape
    bufA = bytearray(np.ascontiguousarray(A, dtype=np.uint32).tobytes())
    C = np.zeros((2, n, n), dtype=np.uint32)
    bufC = bytearray(C.tobytes())
    bufW = bytearray(max(plan.ws, 16))
    rng = np.random.default_rng(4321)
    bufW[:] = rng.integers(0, 256, size=len(bufW), dtype=np.uint8).tobytes()
    sim = Sim([bufA, bufC, bufW], p, plan)
    sim.run(order)
    return np.frombuffer(bytes(bufC), dtype=np.uint32).reshape(2, n, n).copy()


def simulate(plan_text: str, p: int, A_bytes: bytes, C: np.ndarray, order=None) -> np.ndarray:
    """Run the schedule on host copies (in program order, or in the given
    order of operation indices); returns the resulting C (uint32)."""
    plan = parse(plan_text)
    bufA = bytearray(A_bytes)
    bufC = bytearray(np.ascontiguousarray(C, dtype=np.uint32).tobytes())
    bufW = bytearray(max(plan.ws, 16))
    # garbage in the workspace: a schedule must never read what it did not write
    rng = np.random.default_rng(12345)
    bufW[:] = rng.integers(0, 256, size=len(bufW), dtype=np.uint8).tobytes()
    sim = Sim([bufA, bufC, bufW], p, plan)
    sim.run(order)
    return np.frombuffer(bytes(bufC), dtype=np.uint32).reshape(C.shape).copy()
