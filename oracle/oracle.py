"""Plain FP64 CPU oracle for the surrogate-matrix IGA path.

TEST INFRASTRUCTURE ONLY.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import this module.  The product (the HIP
library and its Python binding) never calls it, and it calls nothing of the
product: it shares no code, header, table or constant with the GPU path.

It follows Drzisga, Keith & Wohlmuth, "The surrogate matrix methodology:
Low-cost assembly for isogeometric analysis":

* exact rows and the load vector come from ``igs_oracle.c`` (row-wise Gauss
  quadrature of eq. BilinearFormPoissonTensor, Sec. 3.2, and of the mass form);
* the surrogate follows Sec. 4.1 (tensor B-spline interpolation of every
  stencil function on the sample lattice, Sec. 6 on existing IGA
  codes) and Sec. 5: eq. DefinitionOfSurrogateMatrixSymmetricKernel (5.1c)
  for stiffness, eq. DefinitionOfSurrogateMatrixSymmetric (5.1b) for mass;
* the solve eliminates Dirichlet dofs as in the remark on Dirichlet boundary
  conditions (Sec. 6, eq. BlockSystem) and runs plain conjugate gradients;
* the compliance gradient is -u^T (dA~/dc_k) u, with dA~/dc_k obtained by
  pushing the derivative of the exact entries through the same (linear)
  surrogate construction.

Readings of points the paper leaves open (quadrature rule, interpolation
knots, sample-lattice end rule, which rows use quadrature, diagonal scope)
are the ones listed in the design notes; each function states the one it uses.
"""
from __future__ import annotations

import ctypes
import math
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "igs_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

GEOM = {"identity": 0, "sine": 1, "poly2": 2}
COEF = {"const": 0, "sine3": 1, "spline": 2, "exp_spline": 3}
STIFFNESS, MASS = 0, 1


def build(force: bool = False) -> str:
    """Compile the C half of the oracle with gcc (-O2, OpenMP)."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-o", tmp, _SRC, "-lm"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is None:
        build()
        lib = ctypes.CDLL(_LIB_PATH)
        i32p = ctypes.POINTER(ctypes.c_int32)
        f64p = ctypes.POINTER(ctypes.c_double)
        i64p = ctypes.POINTER(ctypes.c_int64)
        lib.or_gauss.argtypes = [ctypes.c_int, f64p, f64p]
        lib.or_basis.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, f64p, f64p]
        lib.or_rows.argtypes = [i32p, f64p, f64p, ctypes.c_int, ctypes.c_int, i64p, ctypes.c_int64, f64p]
        lib.or_rhs.argtypes = [i32p, f64p, f64p, ctypes.c_int, ctypes.c_double, i64p, ctypes.c_int64, f64p]
        lib.or_map.argtypes = [i32p, f64p, f64p, ctypes.c_int64, f64p, f64p]
        lib.or_threads.argtypes = []
        _lib = lib
    return _lib


def threads():
    """OpenMP threads used by the C half of the oracle."""
    return int(_load().or_threads())


def _ptr(a, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


# --------------------------------------------------------------- problem ----
def dims(prob):
    """m_d = nelem_d + p functions per direction, N = prod m_d, S_st = (2p+1)^n."""
    n, p = prob["n"], prob["p"]
    m = tuple(int(prob["nelem"][d]) + p for d in range(n))
    return m, int(np.prod(m)), (2 * p + 1) ** n


def _params(prob, b=0):
    n, p = prob["n"], prob["p"]
    ne = list(prob["nelem"]) + [1] * (3 - n)
    cn = list(prob.get("cn", (0,) * n)) + [1] * (3 - n)
    ip = np.array([n, p, ne[0], ne[1], ne[2], prob.get("nq", 0), GEOM[prob.get("geom", "identity")],
                   COEF[prob.get("coef", "const")], prob.get("cdeg", 0), cn[0], cn[1], cn[2]], dtype=np.int32)
    dp = np.array([prob.get("ga", 0.0), prob.get("c0", 1.0), prob.get("camp", 0.0)], dtype=np.float64)
    cc = prob.get("cc")
    if cc is not None:
        cc = np.ascontiguousarray(np.asarray(cc, dtype=np.float64).reshape(prob.get("batch", 1), -1)[b])
    else:
        cc = np.zeros(1)
    return ip, dp, cc


def gauss(nq):
    x, w = np.zeros(nq), np.zeros(nq)
    if _load().or_gauss(nq, _ptr(x, ctypes.c_double), _ptr(w, ctypes.c_double)):
        raise ValueError("bad quadrature order")
    return x, w


def basis(nelem, p, k, x):
    """Value and derivative of the k-th (0-based) open-uniform B-spline at x."""
    v, d = ctypes.c_double(), ctypes.c_double()
    _load().or_basis(nelem, p, k, x, ctypes.byref(v), ctypes.byref(d))
    return v.value, d.value


def exact_rows(prob, form, rows, b=0, dcoef=-1):
    """Exact band rows [len(rows), S_st] by element quadrature of row i's support."""
    ip, dp, cc = _params(prob, b)
    rows = np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    _, _, S = dims(prob)
    out = np.zeros((len(rows), S))
    st = _load().or_rows(_ptr(ip, ctypes.c_int32), _ptr(dp, ctypes.c_double), _ptr(cc, ctypes.c_double),
                         form, dcoef, _ptr(rows, ctypes.c_int64), len(rows), _ptr(out, ctypes.c_double))
    if st == -2:
        raise ValueError("geometry map folds: det J <= 0 at a quadrature point")
    if st:
        raise ValueError("oracle rejected the problem")
    return out


def rhs(prob, src, c, b=0, rows=None):
    """Load vector F(B_i) for f = c (src 0) or c prod sin(pi x_d) (src 1)."""
    ip, dp, cc = _params(prob, b)
    _, N, _ = dims(prob)
    rows = np.arange(N, dtype=np.int64) if rows is None else np.ascontiguousarray(np.asarray(rows, dtype=np.int64))
    out = np.zeros(len(rows))
    st = _load().or_rhs(_ptr(ip, ctypes.c_int32), _ptr(dp, ctypes.c_double), _ptr(cc, ctypes.c_double),
                        src, float(c), _ptr(rows, ctypes.c_int64), len(rows), _ptr(out, ctypes.c_double))
    if st:
        raise ValueError("oracle rejected the problem")
    return out


def geometry_map(prob, xi):
    """Physical points F(xi) and det J at parametric points xi [npts, n]."""
    ip, dp, _ = _params(prob)
    xi = np.ascontiguousarray(np.asarray(xi, dtype=np.float64))
    F = np.zeros_like(xi)
    det = np.zeros(len(xi))
    _load().or_map(_ptr(ip, ctypes.c_int32), _ptr(dp, ctypes.c_double), _ptr(xi, ctypes.c_double), len(xi),
                   _ptr(F, ctypes.c_double), _ptr(det, ctypes.c_double))
    return F, det


# ------------------------------------------------------- index helpers -----
def multi_index(prob, rows):
    """Colexicographic multi-index (Sec. 2.2): i = i_1 + m_1 i_2 + m_1 m_2 i_3 (0-based)."""
    m, _, _ = dims(prob)
    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros((len(rows), prob["n"]), dtype=np.int64)
    r = rows.copy()
    for d in range(prob["n"]):
        out[:, d] = r % m[d]
        r //= m[d]
    return out


def flat_index(prob, idx):
    m, _, _ = dims(prob)
    r = np.zeros(idx.shape[0], dtype=np.int64)
    stride = 1
    for d in range(prob["n"]):
        r += idx[:, d] * stride
        stride *= m[d]
    return r


def stencil_offsets(prob):
    """delta for every slot s = sum_d (delta_d + p)(2p+1)^d, delta_1 fastest."""
    n, p = prob["n"], prob["p"]
    w = 2 * p + 1
    S = w ** n
    off = np.zeros((S, n), dtype=np.int64)
    for s in range(S):
        r = s
        for d in range(n):
            off[s, d] = r % w - p
            r //= w
    return off


def interior_mask(prob, idx):
    """Row i lies in the analysis domain (Sec. 4: the intersection of all stencil
    domains) iff every i_d is in [2p, m_d - 2p - 1] (0-based)."""
    m, _, _ = dims(prob)
    p = prob["p"]
    ok = np.ones(idx.shape[0], dtype=bool)
    for d in range(prob["n"]):
        ok &= (idx[:, d] >= 2 * p) & (idx[:, d] <= m[d] - 2 * p - 1)
    return ok


def lattice(m, p, M):
    """Sample indices along one direction (Sec. 6): start at the first analysis
    index 2p, take every M-th index, and append the last index m-2p-1 when M
    does not land on it (the last interval may then be shorter than M)."""
    lo, hi = 2 * p, m - 2 * p - 1
    if hi < lo:
        raise ValueError("no analysis-domain rows: m - 4p < 1")
    s = list(range(lo, hi + 1, M))
    if s[-1] != hi:
        s.append(hi)
    return np.array(s, dtype=np.int64)


def sampling_length(nelem, p, q, c, beta=0.5):
    """Mesh-dependent sampling length of Sec. 7.3.3:
    M(h) = max{1, floor(c h^((p - q + beta)/(q + 1)))}, h = 1/nelem.

    Evaluated exactly in rational arithmetic on the given (binary) values of c
    and beta: M is the largest integer k >= 1 with k <= c' nelem^e',
    e' = (q - p - beta)/(q + 1), c' = c (1 + 1e-12) (the reading: a value
    within 1e-12 relative below an integer counts as that integer).  With
    beta = a/b both sides are raised to the power (q+1) b, which leaves only
    integer powers: k^((q+1)b) <= c'^((q+1)b) nelem^((q-p)b - a)."""
    from fractions import Fraction

    if nelem < 1 or p < 1 or q < 1 or c < 0 or beta < 0:
        raise ValueError("sampling_length: invalid argument")
    fb = Fraction(beta)
    if fb.denominator > 64:
        raise ValueError("sampling_length: beta must have a small binary denominator")
    a, b = fb.numerator, fb.denominator
    power = (q + 1) * b
    cc = Fraction(c) * Fraction(10**12 + 1, 10**12)
    ex = (q - p) * b - a
    rhs = cc**power * (Fraction(nelem) ** ex)

    def fits(k):
        return Fraction(k) ** power <= rhs

    k = 1
    while fits(k + 1):
        k += 1
    return k


def interp_knots(s, q):
    """Knot vector of the degree-q interpolation space on sample abscissae s:
    end knots repeated q+1 times; interior knots are the samples
    s_{(q+1)/2} .. s_{S-1-(q+1)/2} for odd q (not-a-knot) and the midpoints
    (s_k + s_{k+1})/2, k = q/2 .. S-2-q/2, for even q.  Dimension = len(s)."""
    s = np.asarray(s, dtype=np.float64)
    S = len(s)
    if q % 2 == 1:
        inner = s[(q + 1) // 2: S - (q + 1) // 2]
    else:
        inner = 0.5 * (s[q // 2: S - 1 - q // 2] + s[q // 2 + 1: S - q // 2])
    return np.concatenate([np.full(q + 1, s[0]), inner, np.full(q + 1, s[-1])])


def bspline_matrix(t, q, x):
    """Dense collocation matrix B[a, k] = N_{k,q}(x_a) for knot vector t,
    by the Cox-de Boor recursion; the right end point belongs to the last span."""
    t = np.asarray(t, dtype=np.float64)
    x = np.asarray(x, dtype=np.float64)
    nb = len(t) - q - 1
    nspan = len(t) - 1
    B = np.zeros((len(x), nspan))
    last = max(k for k in range(nspan) if t[k] < t[k + 1])
    for k in range(nspan):
        if t[k] < t[k + 1]:
            B[:, k] = (t[k] <= x) & (x < t[k + 1])
    B[x == t[last + 1], last] = 1.0
    for r in range(1, q + 1):
        Bn = np.zeros((len(x), nspan - r))
        for k in range(nspan - r):
            a = np.zeros(len(x))
            if t[k + r] > t[k]:
                a += (x - t[k]) / (t[k + r] - t[k]) * B[:, k]
            if t[k + r + 1] > t[k + 1]:
                a += (t[k + r + 1] - x) / (t[k + r + 1] - t[k + 1]) * B[:, k + 1]
            Bn[:, k] = a
        B = Bn
    assert B.shape[1] == nb
    return B


# --------------------------------------------------------------- surrogate --
class Surrogate:
    """Surrogate matrix of Sec. 5 built from quadrature rows.

    Rows outside the analysis domain and the rows of the sample lattice are
    exact (quadrature).  For every "upper" stencil delta (colex offset > 0;
    also delta = 0 for the mass form) the sample values
    V_delta[k] = A_{s(k), s(k)+delta} are interpolated by the tensor-product
    degree-q spline of ``interp_knots`` (Sec. 4.1), and

      upper entries, i and j = i+delta in the analysis domain: Phi~_delta(i)
      lower entries, both in the analysis domain:           Phi~_{-delta}(j)
      every other off-diagonal entry:                        exact A_ij
      stiffness diagonal of analysis-domain rows:            -sum_{k != i} A~_ik
      mass diagonal of analysis-domain rows:                 Phi~_0(i)

    (eqs. 5.1c and 5.1b).  ``exact`` maps a row list to exact rows; by default
    it is the oracle quadrature, and the gradient check passes a derivative.
    """

    def __init__(self, prob, form, M, q, b=0, exact=None):
        self.prob, self.form, self.M, self.q, self.b = prob, form, M, q, b
        self.exact = exact if exact is not None else (lambda rows: exact_rows(prob, form, rows, b))
        n, p = prob["n"], prob["p"]
        m, N, S = dims(prob)
        self.m, self.N, self.S = m, N, S
        self.sc = (S - 1) // 2
        self.off = stencil_offsets(prob)
        self.samples = [lattice(m[d], p, M) for d in range(n)]
        for d in range(n):
            if len(self.samples[d]) < q + 1:
                raise ValueError("fewer samples than q+1 in a direction")
        self.knots = [interp_knots(self.samples[d], q) for d in range(n)]
        # collocation matrices G_d[k, c] = N_c(s_k) and evaluation matrices over
        # every index of the direction (only analysis-domain rows are used)
        self.G = [bspline_matrix(self.knots[d], q, self.samples[d]) for d in range(n)]
        self.E = []
        for d in range(n):
            x = np.clip(np.arange(m[d], dtype=np.float64), self.samples[d][0], self.samples[d][-1])
            self.E.append(bspline_matrix(self.knots[d], q, x))
        # sample rows (tensor lattice), colex order with direction 1 fastest
        grids = np.meshgrid(*self.samples[::-1], indexing="ij")
        sidx = np.stack([g.ravel() for g in grids[::-1]], axis=1)
        self.sample_rows = flat_index(prob, sidx)
        Vrows = self.exact(self.sample_rows)                      # [nsamp, S]
        shape = tuple(len(self.samples[d]) for d in range(n))[::-1]
        self.upper = [s for s in range(S) if s > self.sc or (form == MASS and s == self.sc)]
        self.coef = {}
        for s in self.upper:
            c = Vrows[:, s].reshape(shape)
            for d in range(n):                                     # solve along each direction
                ax = n - 1 - d
                c = np.moveaxis(c, ax, 0)
                sh = c.shape
                c = np.linalg.solve(self.G[d], c.reshape(sh[0], -1)).reshape(sh)
                c = np.moveaxis(c, 0, ax)
            self.coef[s] = c

    def phi(self, s, idx):
        """Phi~ for upper slot s at multi-indices idx [npts, n]."""
        n = self.prob["n"]
        c = self.coef[s]
        S1 = c.shape[-1]
        R = c.reshape(-1, S1) @ self.E[0][idx[:, 0]].T             # [S_n..S_2, npts]
        if n == 2:
            return np.einsum("jn,nj->n", R, self.E[1][idx[:, 1]])
        S2 = c.shape[1]
        R = R.reshape(c.shape[0], S2, -1)
        R = np.einsum("kjn,nj->kn", R, self.E[1][idx[:, 1]])
        return np.einsum("kn,nk->n", R, self.E[2][idx[:, 2]])

    def rows(self, rows):
        prob = self.prob
        rows = np.asarray(rows, dtype=np.int64)
        idx = multi_index(prob, rows)
        inner = interior_mask(prob, idx)
        out = np.zeros((len(rows), self.S))
        # rows outside the analysis domain are exact
        if (~inner).any():
            out[~inner] = self.exact(rows[~inner])
        ii = np.nonzero(inner)[0]
        if len(ii) == 0:
            return out
        iidx = idx[ii]
        need_exact = np.zeros(len(ii), dtype=bool)
        jin = np.zeros((len(ii), self.S), dtype=bool)
        for s in range(self.S):
            jidx = iidx + self.off[s]
            jin[:, s] = interior_mask(prob, jidx)
            if s != self.sc:
                need_exact |= ~jin[:, s]
        ex = None
        if need_exact.any():
            ex = np.zeros((len(ii), self.S))
            ex[need_exact] = self.exact(rows[ii[need_exact]])
        vals = np.zeros((len(ii), self.S))
        for s in range(self.S):
            if s == self.sc:
                continue
            sel = jin[:, s]
            if s > self.sc:
                vals[sel, s] = self.phi(s, iidx[sel])
            else:
                vals[sel, s] = self.phi(self.S - 1 - s, iidx[sel] + self.off[s])
            if (~sel).any():
                vals[~sel, s] = ex[~sel, s]
        if self.form == STIFFNESS:
            vals[:, self.sc] = -(vals.sum(axis=1) - vals[:, self.sc])
        else:
            vals[:, self.sc] = self.phi(self.sc, iidx)
        out[ii] = vals
        return out


def layer_classes(prob):
    """Row classes of the face/edge stencil functions (Sec. 3.6 reading).

    In direction d an index is "free" when it lies in the analysis range
    [2p, m_d - 2p - 1] (there b_{i_d} and every partner b_{i_d + delta_d} are
    translates of one cardinal B-spline) and otherwise sits in one of the 4p
    boundary layers [0, 2p) u [m_d - 2p, m_d).  The class of row i is the tuple
    key_d = -1 (free) or i_d (its layer); rows of one class are translates of
    each other along the free directions, so every stencil function
    Phi^key_delta is a function of the free coordinates alone.  Returns the
    keys with at least one free direction (interior, faces, edges); the
    classes without one are the corner rows."""
    n, p = prob["n"], prob["p"]
    m, _, _ = dims(prob)
    opts = []
    for d in range(n):
        opts.append([-1] + list(range(2 * p)) + list(range(m[d] - 2 * p, m[d])))
    keys = []
    for key in np.ndindex(*[len(o) for o in opts]):
        k = tuple(opts[d][key[d]] for d in range(n))
        if any(v < 0 for v in k):
            keys.append(k)
    return keys


def row_class(prob, idx):
    """Class keys [npts, n] of multi-indices idx (-1 in free directions)."""
    m, _, _ = dims(prob)
    p = prob["p"]
    key = idx.copy()
    for d in range(prob["n"]):
        free = (idx[:, d] >= 2 * p) & (idx[:, d] <= m[d] - 2 * p - 1)
        key[free, d] = -1
    return key


class SurrogateFE:
    """Surrogate with face- and edge-based stencil functions (Sec. 3.6: a
    family of stencil functions for each face and edge, exploiting the
    translation invariance that remains parallel to them).

    Reading (the paper states the idea only):
      * classes as in ``layer_classes``; each class with at least one free
        direction has, for every upper delta (colex offset > 0; also delta = 0
        for the mass form), its own stencil function over its free
        coordinates, sampled on the tensor lattice of the free directions
        (the same 1-D lattice as the analysis domain, Sec. 6) at the class's
        fixed layers, and interpolated by the degree-q tensor spline of
        ``interp_knots`` (Sec. 4.1) along the free directions only;
      * rows with no free direction (corners) are exact (quadrature);
      * entries, extending eq. 5.1c to the classes: for i < j the value is
        decided by the smaller index i, Phi~^{c(i)}_delta(i) when row i has a
        free direction, else the exact A_ij; for i > j it is the value of
        the pair (j, i) (symmetry); entries whose partner leaves the index box
        are 0;
      * stiffness: every diagonal is -sum_{k != i} A~_ik (eq. 5.1c as stated,
        for every row); mass: the diagonal is interpolated (delta = 0 is an
        upper stencil, eq. 5.1b), exact on corner rows.
    Lower entries whose smaller partner is a corner row take row i's own
    quadrature here; the GPU copies A_ji from the partner (equal to rounding).
    """

    def __init__(self, prob, form, M, q, b=0, exact=None):
        self.prob, self.form, self.M, self.q, self.b = prob, form, M, q, b
        self.exact = exact if exact is not None else (lambda rows: exact_rows(prob, form, rows, b))
        n, p = prob["n"], prob["p"]
        m, N, S = dims(prob)
        self.m, self.N, self.S = m, N, S
        self.sc = (S - 1) // 2
        self.off = stencil_offsets(prob)
        self.samples = [lattice(m[d], p, M) for d in range(n)]
        for d in range(n):
            if len(self.samples[d]) < q + 1:
                raise ValueError("fewer samples than q+1 in a direction")
        knots = [interp_knots(self.samples[d], q) for d in range(n)]
        self.G = [bspline_matrix(knots[d], q, self.samples[d]) for d in range(n)]
        self.E = []
        for d in range(n):
            x = np.clip(np.arange(m[d], dtype=np.float64), self.samples[d][0], self.samples[d][-1])
            self.E.append(bspline_matrix(knots[d], q, x))
        self.upper = [s for s in range(S) if s > self.sc or (form == MASS and s == self.sc)]
        self.keys = layer_classes(prob)
        # sample rows of every class, then one batch of exact rows for all
        srows, spans = [], {}
        for key in self.keys:
            sets = [self.samples[d] if key[d] < 0 else np.array([key[d]]) for d in range(n)]
            g = np.meshgrid(*sets[::-1], indexing="ij")
            r = flat_index(prob, np.stack([x.ravel() for x in g[::-1]], axis=1))
            spans[key] = (sum(len(x) for x in srows), len(r), tuple(len(x) for x in sets)[::-1])
            srows.append(r)
        self.sample_rows = np.concatenate(srows)
        V = self.exact(self.sample_rows)
        self.coef = {}
        for key in self.keys:
            start, cnt, shape = spans[key]
            free = [d for d in range(n) if key[d] < 0]
            for s in self.upper:
                c = V[start:start + cnt, s].reshape(shape)
                for d in free:                                    # solve along each free direction
                    ax = n - 1 - d
                    c = np.moveaxis(c, ax, 0)
                    sh = c.shape
                    c = np.linalg.solve(self.G[d], c.reshape(sh[0], -1)).reshape(sh)
                    c = np.moveaxis(c, 0, ax)
                self.coef[(key, s)] = c

    def phi(self, key, s, idx):
        """Phi~^key for upper slot s at multi-indices idx [npts, n] of rows of
        class key (only their free coordinates enter)."""
        n = self.prob["n"]
        c = self.coef[(key, s)]
        v = c.reshape(c.shape + (1,)) * np.ones(len(idx))             # [..., npts]
        for d in range(n):                                            # contract the last axis first (direction 1)
            ax = n - 1 - d
            if key[d] < 0:
                w = self.E[d][idx[:, d]]                                  # [npts, S_d]
                v = np.einsum("...jn,nj->...n", np.moveaxis(v, ax, -2), w)
            else:
                v = np.moveaxis(v, ax, -2)[..., 0, :]
        return v.reshape(len(idx))

    def rows(self, rows):
        prob = self.prob
        n = prob["n"]
        rows = np.asarray(rows, dtype=np.int64)
        idx = multi_index(prob, rows)
        key = row_class(prob, idx)
        corner = np.all(key >= 0, axis=1)
        mvec = np.array(self.m)
        out = np.zeros((len(rows), self.S))
        ex = self.exact(rows)                       # exact values: corner rows and corner partners
        for s in range(self.S):
            jidx = idx + self.off[s]
            inbox = np.all((jidx >= 0) & (jidx < mvec), axis=1)
            if s == self.sc and self.form == STIFFNESS:
                continue
            if s in self.upper:
                own, part = ~corner & inbox, None
                sel, src_idx, src_key, slot = own, idx, key, s
            else:
                jkey = row_class(prob, np.where(inbox[:, None], jidx, 0))
                jcorner = np.all(jkey >= 0, axis=1)
                sel, src_idx, src_key, slot = inbox & ~jcorner, jidx, jkey, self.S - 1 - s
            val = np.where(inbox, ex[:, s], 0.0)
            ii = np.nonzero(sel)[0]
            if len(ii):
                ks = src_key[ii]
                for kk in np.unique(ks, axis=0):
                    grp = ii[np.all(ks == kk, axis=1)]
                    val[grp] = self.phi(tuple(int(v) for v in kk), slot, src_idx[grp])
            out[:, s] = val
        if self.form == STIFFNESS:
            out[:, self.sc] = -(out.sum(axis=1) - out[:, self.sc])
        return out


def surrogate_rows(prob, form, M, q, rows=None, b=0):
    _, N, _ = dims(prob)
    rows = np.arange(N) if rows is None else rows
    return Surrogate(prob, form, M, q, b).rows(rows)


def surrogate_fe_rows(prob, form, M, q, rows=None, b=0):
    _, N, _ = dims(prob)
    rows = np.arange(N) if rows is None else rows
    return SurrogateFE(prob, form, M, q, b).rows(rows)


def quadrature_rows_fe(prob, M):
    """Rows the face/edge surrogate assembles by quadrature: the sample rows of
    every class with a free direction, plus the corner rows."""
    m, N, _ = dims(prob)
    p = prob["p"]
    idx = multi_index(prob, np.arange(N))
    key = row_class(prob, idx)
    out = np.all(key >= 0, axis=1)
    samp = np.ones(N, dtype=bool)
    for d in range(prob["n"]):
        samp &= (key[:, d] >= 0) | np.isin(idx[:, d], lattice(m[d], p, M))
    return out | samp


def quadrature_rows(prob, M):
    """Rows the surrogate assembles by quadrature: every row outside the analysis
    domain plus the sample lattice."""
    m, N, _ = dims(prob)
    idx = multi_index(prob, np.arange(N))
    out = ~interior_mask(prob, idx)
    samp = np.ones(N, dtype=bool)
    for d in range(prob["n"]):
        samp &= np.isin(idx[:, d], lattice(m[d], prob["p"], M))
    return out | samp


# ----------------------------------------------------- per-delta domains ---
def cardinal_range(m, p):
    """Indices of the cardinal B-splines along one direction (0-based): those
    whose support spans p+1 uniform knot intervals, [p, m - p - 1]."""
    return p, m - p - 1


def delta_range(m, p, dd):
    """Index range of the domain of the stencil function for offset dd along one
    direction (Sec. 4, the remark after the analysis domain): rows i whose own
    function and partner i + dd are both cardinal,
    [p + max(0, -dd), m - p - 1 - max(0, dd)]."""
    return p + max(0, -dd), m - p - 1 - max(0, dd)


def lattice_pd(m, p, M, dd):
    """Sample indices of the stencil function for offset dd along one direction
    (reading): the analysis-domain lattice (``lattice``) plus every index of
    the two transition bands [p, 2p) and (m - 2p - 1, m - p - 1] that lies in
    ``delta_range``; in index order.  Every offset draws on one common set of
    sample indices (lattice plus both bands), and M = 1 samples every index."""
    lo, hi = delta_range(m, p, dd)
    base = lattice(m, p, M)
    s = list(range(lo, 2 * p)) + list(base) + list(range(m - 2 * p, hi + 1))
    return np.array(s, dtype=np.int64)


def sample_union_pd(m, p, M):
    """The common sample indices of every offset along one direction."""
    return np.unique(np.concatenate([lattice_pd(m, p, M, dd) for dd in range(-p, p + 1)]))


def cardinal_mask(prob, idx):
    m, _, _ = dims(prob)
    p = prob["p"]
    ok = np.ones(idx.shape[0], dtype=bool)
    for d in range(prob["n"]):
        lo, hi = cardinal_range(m[d], p)
        ok &= (idx[:, d] >= lo) & (idx[:, d] <= hi)
    return ok


class SurrogatePD:
    """Surrogate with a domain per stencil function (Sec. 4: the results hold
    with the analysis domain replaced by the domain of each stencil function,
    given an interpolation operator per offset; Sec. 5.1-5.3 for the entries).

    Reading:
      * the domain of Phi_delta is the tensor product of ``delta_range``:
        rows i such that i and i + delta index cardinal B-splines;
      * Phi_delta (upper delta: colex offset > 0, also delta = 0 for the mass
        form) is sampled on the tensor product of ``lattice_pd`` and
        interpolated by the degree-q tensor spline of ``interp_knots``;
      * entries: upper delta with i + delta cardinal (i cardinal):
        Phi~_delta(i); lower delta with both cardinal: Phi~_{-delta}(i + delta)
        (eq. 5.1b); every other entry exact (at least one function is not
        cardinal), 0 outside the index box;
      * stiffness diagonal of cardinal rows: -sum_{k != i} A~_ik (eq. 5.1c);
        mass diagonal of cardinal rows: Phi~_0(i); rows of non-cardinal
        functions are exact.
    Quadrature rows: the non-cardinal rows and the tensor product of
    ``sample_union_pd``.
    """

    def __init__(self, prob, form, M, q, b=0, exact=None):
        self.prob, self.form, self.M, self.q, self.b = prob, form, M, q, b
        self.exact = exact if exact is not None else (lambda rows: exact_rows(prob, form, rows, b))
        n, p = prob["n"], prob["p"]
        m, N, S = dims(prob)
        self.m, self.N, self.S = m, N, S
        self.sc = (S - 1) // 2
        self.off = stencil_offsets(prob)
        self.U = [sample_union_pd(m[d], p, M) for d in range(n)]
        self.samp, self.G, self.E = {}, {}, {}
        for d in range(n):
            for dd in range(-p, p + 1):
                sm = lattice_pd(m[d], p, M, dd)
                if len(sm) < q + 1:
                    raise ValueError("fewer samples than q+1 in a direction")
                kn = interp_knots(sm, q)
                self.samp[(d, dd)] = sm
                self.G[(d, dd)] = bspline_matrix(kn, q, sm)
                x = np.clip(np.arange(m[d], dtype=np.float64), sm[0], sm[-1])
                self.E[(d, dd)] = bspline_matrix(kn, q, x)
        # exact rows at every sample index (tensor product of the unions)
        g = np.meshgrid(*self.U[::-1], indexing="ij")
        uidx = np.stack([x.ravel() for x in g[::-1]], axis=1)
        self.sample_rows = flat_index(prob, uidx)
        V = self.exact(self.sample_rows)
        shapeU = tuple(len(u) for u in self.U)[::-1]
        V = V.reshape(shapeU + (S,))
        self.upper = [s for s in range(S) if s > self.sc or (form == MASS and s == self.sc)]
        self.coef = {}
        for s in self.upper:
            c = V[..., s]
            for d in range(n):                   # restrict to this offset's samples, then solve
                ax = n - 1 - d
                pos = np.searchsorted(self.U[d], self.samp[(d, int(self.off[s, d]))])
                c = np.take(c, pos, axis=ax)
            for d in range(n):
                ax = n - 1 - d
                c = np.moveaxis(c, ax, 0)
                sh = c.shape
                c = np.linalg.solve(self.G[(d, int(self.off[s, d]))], c.reshape(sh[0], -1)).reshape(sh)
                c = np.moveaxis(c, 0, ax)
            self.coef[s] = c

    def phi(self, s, idx):
        """Phi~ for upper slot s at multi-indices idx [npts, n]."""
        n = self.prob["n"]
        c = self.coef[s]
        v = c.reshape(c.shape + (1,)) * np.ones(len(idx))
        for d in range(n):                       # direction 1 is the last axis of c
            w = self.E[(d, int(self.off[s, d]))][idx[:, d]]
            v = np.einsum("...jn,nj->...n", v, w)
        return v.reshape(len(idx))

    def rows(self, rows):
        prob = self.prob
        rows = np.asarray(rows, dtype=np.int64)
        idx = multi_index(prob, rows)
        card = cardinal_mask(prob, idx)
        mvec = np.array(self.m)
        ex = self.exact(rows)
        out = np.zeros((len(rows), self.S))
        for s in range(self.S):
            jidx = idx + self.off[s]
            inbox = np.all((jidx >= 0) & (jidx < mvec), axis=1)
            val = np.where(inbox, ex[:, s], 0.0)
            if s == self.sc:
                if self.form == MASS:
                    ii = np.nonzero(card)[0]
                    val[ii] = self.phi(s, idx[ii])
                out[:, s] = val
                continue
            both = card & inbox & cardinal_mask(prob, np.where(inbox[:, None], jidx, 0))
            ii = np.nonzero(both)[0]
            if len(ii):
                if s > self.sc:
                    val[ii] = self.phi(s, idx[ii])
                else:
                    val[ii] = self.phi(self.S - 1 - s, jidx[ii])
            out[:, s] = val
        if self.form == STIFFNESS:
            ii = np.nonzero(card)[0]
            out[ii, self.sc] = -(out[ii].sum(axis=1) - out[ii, self.sc])
        return out


def surrogate_pd_rows(prob, form, M, q, rows=None, b=0):
    _, N, _ = dims(prob)
    rows = np.arange(N) if rows is None else rows
    return SurrogatePD(prob, form, M, q, b).rows(rows)


def quadrature_rows_pd(prob, M):
    """Rows the per-delta surrogate assembles by quadrature: the rows of
    non-cardinal functions plus the tensor product of the sample unions."""
    m, N, _ = dims(prob)
    p = prob["p"]
    idx = multi_index(prob, np.arange(N))
    samp = np.ones(N, dtype=bool)
    for d in range(prob["n"]):
        samp &= np.isin(idx[:, d], sample_union_pd(m[d], p, M))
    return ~cardinal_mask(prob, idx) | samp


# -------------------------------------------------------- linear algebra ---
def dirichlet_mask(prob):
    """Dofs whose function does not vanish on the boundary: some i_d in {0, m_d-1}."""
    m, N, _ = dims(prob)
    idx = multi_index(prob, np.arange(N))
    D = np.zeros(N, dtype=bool)
    for d in range(prob["n"]):
        D |= (idx[:, d] == 0) | (idx[:, d] == m[d] - 1)
    return D


def to_csr(prob, band_rows):
    """Sparse matrix from band rows [N, S_st] (entries with j out of range are 0)."""
    import scipy.sparse as sp

    m, N, S = dims(prob)
    idx = multi_index(prob, np.arange(N))
    off = stencil_offsets(prob)
    R, C, V = [], [], []
    for s in range(S):
        jidx = idx + off[s]
        ok = np.all((jidx >= 0) & (jidx < np.array(m)), axis=1)
        R.append(np.nonzero(ok)[0])
        C.append(flat_index(prob, jidx[ok]))
        V.append(band_rows[ok, s])
    return sp.csr_matrix((np.concatenate(V), (np.concatenate(R), np.concatenate(C))), shape=(N, N))


def apply(prob, band_rows, x, dirichlet=False):
    """y = A x from band rows; with dirichlet, rows and columns of boundary dofs are dropped (y_D = 0)."""
    A = to_csr(prob, band_rows)
    x = np.array(x, dtype=np.float64)
    if dirichlet:
        D = dirichlet_mask(prob)
        x[D] = 0.0
        y = A @ x
        y[D] = 0.0
        return y
    return A @ x


def cg(prob, band_rows, f, rtol=1e-10, maxit=100000):
    """Conjugate gradients on A_II u_I = f_I (homogeneous Dirichlet), x0 = 0.
    Stops when ||f_I - A_II u_I||_2 <= rtol ||f_I||_2 (recursive residual,
    confirmed with the true residual at exit).  Returns (u, iterations, relres)."""
    A = to_csr(prob, band_rows)
    D = dirichlet_mask(prob)
    I = ~D
    AII = A[I][:, I]
    b = np.asarray(f, dtype=np.float64)[I]
    x = np.zeros_like(b)
    r = b.copy()
    pvec = r.copy()
    rr = r @ r
    nb = math.sqrt(b @ b)
    it = 0
    while math.sqrt(rr) > rtol * nb and it < maxit:
        q = AII @ pvec
        alpha = rr / (pvec @ q)
        x += alpha * pvec
        r -= alpha * q
        rr_new = r @ r
        pvec = r + (rr_new / rr) * pvec
        rr = rr_new
        it += 1
    u = np.zeros(len(D))
    u[I] = x
    relres = np.linalg.norm(b - AII @ x) / nb
    return u, it, relres


def quadratic_form(prob, band_rows, u, v=None):
    """v^T A u from band rows."""
    A = to_csr(prob, band_rows)
    v = u if v is None else v
    return float(v @ (A @ u))


def bilinear_grad(prob, M, q, ybar, x, ks, b=0, surrogate=True):
    """d/dc_k (ybar^T A~(c) x) = ybar^T (dA~/dc_k) x.  dA~/dc_k is the surrogate
    construction (linear in the quadrature values) applied to the exact
    derivative entries dA_ij/dc_k = int dkappa/dc_k grad B_i^T K grad B_j."""
    _, N, _ = dims(prob)
    g = np.zeros(len(ks))
    for t, k in enumerate(ks):
        ex = (lambda rows, k=k: exact_rows(prob, STIFFNESS, rows, b, dcoef=int(k)))
        if surrogate:
            dband = Surrogate(prob, STIFFNESS, M, q, b, exact=ex).rows(np.arange(N))
        else:
            dband = ex(np.arange(N))
        g[t] = quadratic_form(prob, dband, x, ybar)
    return g


def compliance_grad(prob, M, q, u, ks, b=0, surrogate=True):
    """dJ/dc_k for J = f^T u with A~(c) u = f: dJ/dc_k = -u^T (dA~/dc_k) u."""
    return -bilinear_grad(prob, M, q, u, u, ks, b, surrogate)


def l2_error(prob, u, exact_fn, nq=None):
    """Relative L2 error ||u - u_h|| / ||u|| of u_h = sum_i u_i B_i against
    exact_fn(x) on the physical domain, by Gauss quadrature on every element."""
    n, p = prob["n"], prob["p"]
    m, N, _ = dims(prob)
    nq = nq or p + 2
    gx, gw = gauss(nq)
    pts1d, w1d, Bm = [], [], []
    for d in range(n):
        ne = prob["nelem"][d]
        h = 1.0 / ne
        e = np.arange(ne)[:, None]
        x = ((e + 0.5 * (gx[None, :] + 1.0)) * h).ravel()
        w = np.tile(0.5 * h * gw, ne)
        t = np.concatenate([np.zeros(p + 1), np.arange(1, ne) / ne, np.ones(p + 1)])
        pts1d.append(x)
        w1d.append(w)
        Bm.append(bspline_matrix(t, p, x))
    U = np.asarray(u).reshape([m[d] for d in range(n)][::-1])
    # u_h on the tensor grid of quadrature points
    V = U
    for d in range(n):
        ax = n - 1 - d
        V = np.moveaxis(np.tensordot(Bm[d], np.moveaxis(V, ax, 0), axes=(1, 0)), 0, ax)
    grids = np.meshgrid(*pts1d[::-1], indexing="ij")
    xi = np.stack([g.ravel() for g in grids[::-1]], axis=1)
    W = np.ones(1)
    for d in range(n):
        W = np.multiply.outer(w1d[d], W) if d else w1d[0]
    F, det = geometry_map(prob, xi)
    uh = V.ravel()
    ue = exact_fn(F)
    wt = W.ravel() * np.abs(det)
    return math.sqrt(np.sum(wt * (ue - uh) ** 2) / np.sum(wt * ue ** 2))
