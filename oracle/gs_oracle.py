"""Python bindings of the GridShift FP64 CPU oracle.

TEST INFRASTRUCTURE ONLY.  The oracle is the plain, slow reference the GPU
path is checked against.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import this module.  It shares no code with
the GPU library: it compiles ``gs_oracle.c`` with gcc into
``liboracle_gs.so`` next to this file and calls it through ctypes.

The semantics (GridShift, arXiv 2206.02200, Section 2.1 and Algorithm 1, in
the parallel update form of Eq. 6) are documented at the top of
``gs_oracle.c``.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "gs_oracle.c")
# GS_ORACLE_SANITIZE=1 selects an AddressSanitizer + UndefinedBehaviorSanitizer
# build (liboracle_gs_san.so); the process must then preload the sanitizer
# runtimes (oracle/run_sanitized_tests.sh does).
SANITIZE = os.environ.get("GS_ORACLE_SANITIZE", "") not in ("", "0")
LIB_PATH = os.path.join(_HERE, "liboracle_gs_san.so" if SANITIZE else "liboracle_gs.so")
SANITIZE_FLAGS = ["-g", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
                  "-fno-sanitize-recover=undefined"]

CONVERGED = 1
STATIONARY = 2
CAPPED = 4

_ERRORS = {
    1: "invalid argument",
    2: "non-finite input",
    3: "cell key out of range",
    4: "out of memory",
}


class OracleError(RuntimeError):
    def __init__(self, code: int):
        super().__init__(f"oracle error {code}: {_ERRORS.get(code, 'unknown')}")
        self.code = code


def build(sanitize: bool | None = None) -> str:
    """Compile the oracle with gcc (binary64 SSE2 arithmetic, no contraction);
    with sanitize (default: GS_ORACLE_SANITIZE) the ASan + UBSan build."""
    san = SANITIZE if sanitize is None else sanitize
    path = os.path.join(_HERE, "liboracle_gs_san.so" if san else "liboracle_gs.so")
    cmd = [
        "gcc", "-O2", "-std=gnu11", "-ffp-contract=off", "-fno-fast-math",
        "-fno-strict-aliasing", "-shared", "-fPIC", "-Wall", "-Wextra",
        *(SANITIZE_FLAGS if san else []),
        "-o", path + ".tmp", _SRC, "-lm",
    ]
    subprocess.run(cmd, check=True)
    os.replace(path + ".tmp", path)
    return path


_lib = None


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        build()
    lib = ctypes.CDLL(LIB_PATH)
    P = ctypes.c_void_p
    lib.gso_pairwise_sum.restype = ctypes.c_double
    lib.gso_pairwise_sum.argtypes = [P, ctypes.c_int64]
    lib.gso_bin.restype = ctypes.c_int
    lib.gso_bin.argtypes = [P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P, P, P, P, P]
    lib.gso_has_neighbours.restype = ctypes.c_int
    lib.gso_has_neighbours.argtypes = [P, ctypes.c_int64, ctypes.c_int32]
    lib.gso_shift.restype = None
    lib.gso_shift.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, P, P]
    lib.gso_merge.restype = ctypes.c_int
    lib.gso_merge.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P, P, P, P, P]
    lib.gso_fit_tape.restype = ctypes.c_int
    lib.gso_fit_tape.argtypes = [
        P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
        P, P, P, P, P, P, P, P, P, ctypes.POINTER(P),
    ]
    lib.gso_tape_free.restype = None
    lib.gso_tape_free.argtypes = [P]
    lib.gso_tape_sizes.restype = None
    lib.gso_tape_sizes.argtypes = [P, P, P, P, P]
    lib.gso_tape_round_cells.restype = ctypes.c_int64
    lib.gso_tape_round_cells.argtypes = [P, ctypes.c_int32]
    lib.gso_tape_round.restype = None
    lib.gso_tape_round.argtypes = [P, ctypes.c_int32, P, P, P, P]
    lib.gso_tape_points.restype = None
    lib.gso_tape_points.argtypes = [P, P, P]
    lib.gso_tape_adjoint.restype = ctypes.c_int
    lib.gso_tape_adjoint.argtypes = [P, P, P]
    lib.gso_tape_cluster_sums.restype = ctypes.c_int
    lib.gso_tape_cluster_sums.argtypes = [P, P]
    lib.gso_point_mode_loss.restype = ctypes.c_double
    lib.gso_point_mode_loss.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P, P]
    lib.gso_tape_fd_q.restype = ctypes.c_int
    lib.gso_tape_fd_q.argtypes = [P, P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, P]
    lib.gso_tape_replay_loss.restype = ctypes.c_int
    lib.gso_tape_replay_loss.argtypes = [P, P, P, P]
    lib.gso_fit.restype = ctypes.c_int
    lib.gso_fit.argtypes = [
        P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32,
        P, P, P, P, P, P, P, P, P,
    ]
    lib.gso_fit_rule.restype = ctypes.c_int
    lib.gso_fit_rule.argtypes = [
        P, ctypes.c_int64, ctypes.c_int32, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
        P, P, P, P, P, P, P, P, P,
    ]
    lib.gso_shift_seq.restype = ctypes.c_int
    lib.gso_shift_seq.argtypes = [P, P, P, ctypes.c_int64, ctypes.c_int32, P, P, P]
    lib.gso_colour_order.restype = None
    lib.gso_colour_order.argtypes = [P, ctypes.c_int64, ctypes.c_int32, P]
    _lib = lib
    return lib


def ensure_loaded() -> None:
    """Load (building if needed) the oracle library now, e.g. before several
    host threads start calling it."""
    _load()


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def pairwise_sum(a) -> float:
    """R(a_0..a_{L-1}): a_0 if L == 1, else R(first P) + R(rest), P the largest
    power of two below L."""
    a = np.ascontiguousarray(a, dtype=np.float64)
    return _load().gso_pairwise_sum(_ptr(a), a.size)


@dataclass
class OracleResult:
    labels: np.ndarray  # int32 [n]
    modes: np.ndarray  # float64 [K, d]
    counts: np.ndarray  # int64 [K]
    sums: np.ndarray  # float64 [K, d]
    keys: np.ndarray  # int64 [K, d]
    m_hist: np.ndarray  # int64 [n_iter + 1]: active cells before each round
    K: int
    n_iter: int
    flags: int


# update rules of the shift (gso_fit_rule)
RULES = {"parallel": 0, "sequential_key": 1, "sequential": 2}


def fit(x, h: float, max_iter: int = 100, rule: str = "parallel") -> OracleResult:
    """Run GridShift on points ``x`` ([n, d]; float32 is widened exactly).

    ``rule``: "parallel" (Eq. 6, every cell reads the round's table),
    "sequential" (Eq. 5, cells visited colour by colour: ascending colour,
    the colour's bit d-1-k being the parity of integer coordinate k, then
    ascending key) or "sequential_key" (Eq. 5, cells visited in ascending
    key)."""
    x = np.asarray(x)
    if x.ndim != 2:
        raise ValueError("x must be [n, d]")
    xd = np.ascontiguousarray(x, dtype=np.float64)
    n, d = xd.shape
    cap = max(n, 1)
    labels = np.empty(cap, np.int32)
    modes = np.empty((cap, d), np.float64)
    counts = np.empty(cap, np.int64)
    sums = np.empty((cap, d), np.float64)
    keys = np.empty((cap, d), np.int64)
    m_hist = np.zeros(max_iter + 2, np.int64)
    K = ctypes.c_int64(0)
    T = ctypes.c_int32(0)
    flags = ctypes.c_uint32(0)
    if rule not in RULES:
        raise ValueError(f"unknown rule {rule!r}")
    rc = _load().gso_fit_rule(
        _ptr(xd), n, d, float(h), int(max_iter), RULES[rule],
        _ptr(labels), _ptr(modes), _ptr(counts), _ptr(sums), _ptr(keys), _ptr(m_hist),
        ctypes.byref(K), ctypes.byref(T), ctypes.byref(flags),
    )
    if rc != 0:
        raise OracleError(rc)
    k = K.value
    return OracleResult(
        labels=labels[:n].copy(), modes=modes[:k].copy(), counts=counts[:k].copy(),
        sums=sums[:k].copy(), keys=keys[:k].copy(), m_hist=m_hist[: T.value + 1].copy(),
        K=k, n_iter=T.value, flags=flags.value,
    )


# --------------------------------------------------------------------------
# the individual steps, exposed so that tests can pin each one
# --------------------------------------------------------------------------
@dataclass
class CellTable:
    keys: np.ndarray  # int64 [m, d], ascending lexicographic
    counts: np.ndarray  # int64 [m]
    sums: np.ndarray  # float64 [m, d]


def bin_points(x, h: float) -> tuple[CellTable, np.ndarray]:
    """Section 2.1 (i): cells of side h, counts, R-sums; returns (table, cell0)."""
    xd = np.ascontiguousarray(np.asarray(x), dtype=np.float64)
    n, d = xd.shape
    cap = max(n, 1)
    keys = np.empty((cap, d), np.int64)
    counts = np.empty(cap, np.int64)
    sums = np.empty((cap, d), np.float64)
    cell0 = np.empty(cap, np.int64)
    m = ctypes.c_int64(0)
    rc = _load().gso_bin(_ptr(xd), n, d, float(h), _ptr(keys), _ptr(counts), _ptr(sums), _ptr(cell0),
                         ctypes.byref(m))
    if rc != 0:
        raise OracleError(rc)
    k = m.value
    return CellTable(keys[:k].copy(), counts[:k].copy(), sums[:k].copy()), cell0[:n].copy()


def has_neighbours(table: CellTable) -> bool:
    """Section 2.1 (v): does any active cell have an active neighbour?"""
    keys = np.ascontiguousarray(table.keys, dtype=np.int64)
    m, d = keys.shape
    return bool(_load().gso_has_neighbours(_ptr(keys), m, d))


def shift(table: CellTable) -> tuple[np.ndarray, np.ndarray]:
    """Eq. 1-2 (parallel form, Eq. 6): returns (p [m, d], W [m])."""
    keys = np.ascontiguousarray(table.keys, dtype=np.int64)
    counts = np.ascontiguousarray(table.counts, dtype=np.int64)
    sums = np.ascontiguousarray(table.sums, dtype=np.float64)
    m, d = keys.shape
    p = np.empty((max(m, 1), d), np.float64)
    W = np.empty(max(m, 1), np.int64)
    _load().gso_shift(_ptr(keys), _ptr(counts), _ptr(sums), m, d, _ptr(p), _ptr(W))
    return p[:m].copy(), W[:m].copy()


def colour_order(table: CellTable) -> np.ndarray:
    """Visiting order of the sequential sweep used on the device: ascending
    colour (bit d-1-k = parity of integer coordinate k), then ascending key."""
    keys = np.ascontiguousarray(table.keys, dtype=np.int64)
    m, d = keys.shape
    order = np.empty(max(m, 1), np.int64)
    _load().gso_colour_order(_ptr(keys), m, d, _ptr(order))
    return order[:m].copy()


def shift_sequential(table: CellTable, order) -> tuple[np.ndarray, np.ndarray]:
    """Eq. 5 (sequential form): cells visited in ``order`` (a permutation of
    the table's rows); a visited cell's fl(C * p) replaces its sum for the
    cells visited after it.  Returns (p [m, d], W [m])."""
    keys = np.ascontiguousarray(table.keys, dtype=np.int64)
    counts = np.ascontiguousarray(table.counts, dtype=np.int64)
    sums = np.ascontiguousarray(table.sums, dtype=np.float64)
    order = np.ascontiguousarray(order, dtype=np.int64)
    m, d = keys.shape
    if sorted(order.tolist()) != list(range(m)):
        raise ValueError("order must be a permutation of the table's rows")
    p = np.empty((max(m, 1), d), np.float64)
    W = np.empty(max(m, 1), np.int64)
    rc = _load().gso_shift_seq(_ptr(keys), _ptr(counts), _ptr(sums), m, d, _ptr(order), _ptr(p), _ptr(W))
    if rc != 0:
        raise OracleError(rc)
    return p[:m].copy(), W[:m].copy()


def merge(counts, p, h: float) -> tuple[CellTable, np.ndarray]:
    """Section 2.1 (iii)-(iv), Eq. 3-4: returns (new table, g [m])."""
    counts = np.ascontiguousarray(counts, dtype=np.int64)
    p = np.ascontiguousarray(p, dtype=np.float64)
    m, d = p.shape
    cap = max(m, 1)
    nkeys = np.empty((cap, d), np.int64)
    ncounts = np.empty(cap, np.int64)
    nsums = np.empty((cap, d), np.float64)
    g = np.empty(cap, np.int64)
    nm = ctypes.c_int64(0)
    rc = _load().gso_merge(_ptr(counts), _ptr(p), m, d, float(h), _ptr(nkeys), _ptr(ncounts), _ptr(nsums),
                           _ptr(g), ctypes.byref(nm))
    if rc != 0:
        raise OracleError(rc)
    k = nm.value
    return CellTable(nkeys[:k].copy(), ncounts[:k].copy(), nsums[:k].copy()), g[:m].copy()


# --------------------------------------------------------------------------
# differentiable form: trajectory tape, adjoint, point-to-mode loss
# --------------------------------------------------------------------------
class Tape:
    """Discrete trajectory of one fit (owned C object; see gs_oracle.c)."""

    def __init__(self, handle):
        self._h = handle
        lib = _load()
        n, m0, d, T = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32(), ctypes.c_int32()
        lib.gso_tape_sizes(handle, ctypes.byref(n), ctypes.byref(m0), ctypes.byref(d), ctypes.byref(T))
        self.n, self.m0, self.d, self.T = n.value, m0.value, d.value, T.value
        self.cell0 = np.empty(max(self.n, 1), np.int64)
        self.sums0 = np.empty((max(self.m0, 1), self.d), np.float64)
        if self.n:
            lib.gso_tape_points(handle, _ptr(self.cell0), _ptr(self.sums0))
        self.cell0 = self.cell0[: self.n]
        self.sums0 = self.sums0[: self.m0]
        self.rounds = []
        for t in range(self.T + 1):
            m = lib.gso_tape_round_cells(handle, t)
            keys = np.empty((max(m, 1), self.d), np.int64)
            counts = np.empty(max(m, 1), np.int64)
            W = np.empty(max(m, 1), np.int64)
            g = np.empty(max(m, 1), np.int64)
            if m:
                lib.gso_tape_round(handle, t, _ptr(keys), _ptr(counts), _ptr(W), _ptr(g))
            self.rounds.append({"keys": keys[:m], "counts": counts[:m], "W": W[:m], "g": g[:m]})

    def same_trajectory(self, other: "Tape") -> bool:
        """Identical discrete path: initial cells, and every round's keys,
        counts, weights and merge maps."""
        if (self.n, self.m0, self.d, self.T) != (other.n, other.m0, other.d, other.T):
            return False
        if not np.array_equal(self.cell0, other.cell0):
            return False
        for a, b in zip(self.rounds, other.rounds):
            for f in ("keys", "counts", "W", "g"):
                if not np.array_equal(a[f], b[f]):
                    return False
        return True

    def adjoint(self, mubar) -> np.ndarray:
        """Sbar^0 [m0, d] for a mode cotangent mubar [K, d]."""
        mubar = np.ascontiguousarray(mubar, dtype=np.float64)
        out = np.zeros((max(self.m0, 1), self.d), np.float64)
        rc = _load().gso_tape_adjoint(self._h, _ptr(mubar), _ptr(out))
        if rc:
            raise OracleError(rc)
        return out[: self.m0]

    def point_adjoint(self, mubar) -> np.ndarray:
        """Gradient of sum(mubar * modes) with respect to the points [n, d]."""
        return self.adjoint(mubar)[self.cell0]

    def cluster_point_sums(self) -> np.ndarray:
        """[K, d]: sum of the points of every final cluster (R over initial cells)."""
        K = len(self.rounds[-1]["counts"])
        X = np.zeros((max(K, 1), self.d), np.float64)
        rc = _load().gso_tape_cluster_sums(self._h, _ptr(X))
        if rc:
            raise OracleError(rc)
        return X[:K]

    def fd_q(self, x, i: int, k: int, eps: float) -> float:
        """binary128 central difference of the replayed loss in x[i, k]."""
        xd = np.ascontiguousarray(x, dtype=np.float64)
        out = ctypes.c_double()
        rc = _load().gso_tape_fd_q(self._h, _ptr(xd), int(i), int(k), float(eps), ctypes.byref(out))
        if rc:
            raise OracleError(rc)
        return out.value

    def replay_loss(self, x) -> float:
        xd = np.ascontiguousarray(x, dtype=np.float64)
        hi, lo = ctypes.c_double(), ctypes.c_double()
        rc = _load().gso_tape_replay_loss(self._h, _ptr(xd), ctypes.byref(hi), ctypes.byref(lo))
        if rc:
            raise OracleError(rc)
        return hi.value + lo.value

    def __del__(self):
        h = getattr(self, "_h", None)
        lib = _lib
        if h and lib is not None:
            try:
                lib.gso_tape_free(h)
            except Exception:
                pass
            self._h = None


def fit_tape(x, h: float, max_iter: int = 100) -> tuple[OracleResult, Tape]:
    """fit() that also records the trajectory tape."""
    x = np.asarray(x)
    xd = np.ascontiguousarray(x, dtype=np.float64)
    n, d = xd.shape
    cap = max(n, 1)
    labels = np.empty(cap, np.int32)
    modes = np.empty((cap, d), np.float64)
    counts = np.empty(cap, np.int64)
    sums = np.empty((cap, d), np.float64)
    keys = np.empty((cap, d), np.int64)
    m_hist = np.zeros(max_iter + 2, np.int64)
    K = ctypes.c_int64(0)
    T = ctypes.c_int32(0)
    flags = ctypes.c_uint32(0)
    h_tape = ctypes.c_void_p()
    rc = _load().gso_fit_tape(
        _ptr(xd), n, d, float(h), int(max_iter),
        _ptr(labels), _ptr(modes), _ptr(counts), _ptr(sums), _ptr(keys), _ptr(m_hist),
        ctypes.byref(K), ctypes.byref(T), ctypes.byref(flags), ctypes.byref(h_tape),
    )
    if rc != 0:
        raise OracleError(rc)
    k = K.value
    res = OracleResult(
        labels=labels[:n].copy(), modes=modes[:k].copy(), counts=counts[:k].copy(),
        sums=sums[:k].copy(), keys=keys[:k].copy(), m_hist=m_hist[: T.value + 1].copy(),
        K=k, n_iter=T.value, flags=flags.value,
    )
    return res, Tape(h_tape)


def point_mode_loss(x, labels, modes) -> float:
    """L = R over points (ascending) of the left fold over k of (x_ik - mu)^2."""
    xd = np.ascontiguousarray(x, dtype=np.float64)
    lab = np.ascontiguousarray(labels, dtype=np.int32)
    md = np.ascontiguousarray(modes, dtype=np.float64)
    n, d = xd.shape
    return _load().gso_point_mode_loss(_ptr(xd), n, d, _ptr(lab), _ptr(md))


def loss_and_grad(x, h: float, max_iter: int = 100):
    """Point-to-mode loss and its gradient with the trajectory held fixed:
    grad_i = 2 (x_i - mu_l(i)) + [J^T mubar]_i,  mubar_c = -2 (X_c - C_c mu_c),
    X_c the sum of the points of cluster c."""
    xd = np.ascontiguousarray(np.asarray(x), dtype=np.float64)
    res, tape = fit_tape(xd, h, max_iter)
    L = point_mode_loss(xd, res.labels, res.modes)
    X = tape.cluster_point_sums()
    mubar = -2.0 * (X - res.counts[:, None].astype(np.float64) * res.modes)
    grad = 2.0 * (xd - res.modes[res.labels]) + tape.point_adjoint(mubar)
    return L, grad, res, tape
