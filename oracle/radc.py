"""Spin-adapted, density-fitted EA/IP-ADC(n) on the CPU in FP64 (the oracle).

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
CPU-baseline leg of the benchmark, never by the library.  It shares no code
with the HIP path.

What it computes (Sec. III.A, steps 2-5):
  * amplitudes t (first-order doubles), s, u (second-order singles/doubles),
    w (third-order singles) from Eqs. 13-14 (step 2);
  * the 1p-1p (EA) or 1h-1h (IP) block M11 (step 3);
  * the matrix-vector product sigma = M Y (Eqs. 36-37 and their EA analogue,
    step 4), exact diagonal, explicit M for small cases;
  * spectroscopic amplitudes X = T Y and factors P = 2 sum_p X_p^2
    (Eqs. 16 and 46-50, step 5).
Every two-electron integral is (pq|rs) = sum_Q B^Q_pq B^Q_rs (Eq. 38); the
working equations are the term tables of ``radc_terms`` evaluated one term at
a time with numpy.einsum (no regrouping).

Vector representation used at the library boundary ("Z basis"): the
spin-adapted amplitudes Y of Eqs. 36-37 are not orthonormal; their metric is
S = 1 (+) (2 - P_swap) (the norm of Eq. 48, P_swap exchanging the two like
indices).  The library works with Z = S^{1/2} Y (symmetric square root), an
orthonormal basis of the doublet space, in which M_Z = S^{1/2} M_Y S^{-1/2} is
symmetric.  On each pair (ab, ba):  S^{1/2} = al + be P_swap with
al = (1 + sqrt3)/2, be = (1 - sqrt3)/2, and S^{-1/2} with
al' = (1 + 1/sqrt3)/2, be' = (1 - 1/sqrt3)/2.  Since al + be = 1 the
diagonal a = b is left unchanged.  A normalised Z gives the renormalised
amplitudes of Eqs. 46-48.
Layout of a vector of length dim:
  EA: Z1[a] (V), then Z2[i][a][b] (O*V*V)   (a: attached alpha particle)
  IP: Z1[i] (O), then Z2[a][i][j] (V*O*O)   (i: removed alpha hole)
Eigenvalues: EA omega = E(N+1) - E(N); IP omega = E(N-1) - E(N) > 0 (the IP
matrix is -M_- of Eq. 9).
"""
from __future__ import annotations

import numpy as np
from numpy.lib.stride_tricks import as_strided

from . import radc_terms

SQ3 = np.sqrt(3.0)
AL, BE = (1.0 + SQ3) / 2.0, (1.0 - SQ3) / 2.0            # S^{+1/2}
ALI, BEI = (1.0 + 1.0 / SQ3) / 2.0, (1.0 - 1.0 / SQ3) / 2.0  # S^{-1/2}

OCC_LETTERS = set("ijklmno")


def _space(letter, p_space="v"):
    if letter == "p":
        return p_space
    return "o" if letter in OCC_LETTERS else "v"


def _parse(spec):
    out = []
    for tok in spec.split():
        name, idx = tok.split(":")
        out.append((name, idx))
    return out


class RADC:
    """CPU FP64 spin-adapted ADC(n), n in {2, 3}, kind in {"ea", "ip"}."""

    def __init__(self, eps, B, nocc, order, kind, lazy=False):
        eps = np.asarray(eps, dtype=np.float64)
        B = np.asarray(B, dtype=np.float64)
        if order not in (2, 3) or kind not in ("ea", "ip"):
            raise ValueError("order must be 2 or 3 and kind 'ea' or 'ip'")
        self.order, self.kind = order, kind
        self.O = O = nocc
        self.V = V = eps.size - nocc
        self.eo, self.ev = eps[:O].copy(), eps[O:].copy()
        o, v = slice(0, O), slice(O, O + V)
        self.Bb = {("o", "o"): np.ascontiguousarray(B[:, o, o]),
                   ("o", "v"): np.ascontiguousarray(B[:, o, v]),
                   ("v", "o"): np.ascontiguousarray(B[:, v, o]),
                   ("v", "v"): np.ascontiguousarray(B[:, v, v])}
        self.terms = radc_terms.EA_TERMS if kind == "ea" else radc_terms.IP_TERMS
        self.T = {"f": None}
        self.dim = (V + O * V * V) if kind == "ea" else (O + O * O * V)
        self.n1 = V if kind == "ea" else O
        self._amplitudes()
        self._M11 = None
        if not lazy:            # lazy: third-order amplitudes and M11 on first use
            self._third_order()
            self._M11 = self._m11()

    @property
    def M11(self):
        if self._M11 is None:
            self._third_order()
            self._M11 = self._m11()
        return self._M11

    # ------------------------------------------------------------------
    # term evaluation
    # ------------------------------------------------------------------
    def _operands(self, spec, Y1=None, Y2=None, p_space="v", y1_eye=None):
        """einsum subscripts and operands for one product of tensors.

        Y1/Y2 carry a leading vector index 'z'.  With y1_eye, Y1:x becomes the
        identity with subscripts x + y1_eye (columns of the 11 block).
        """
        subs, ops = [], []
        for name, idx in _parse(spec):
            if name == "g":   # (pq|rs) = sum_Q B^Q_pq B^Q_rs
                p, q, r, s = idx
                subs.append("Q" + p + q)
                ops.append(self.Bb[(_space(p, p_space), _space(q, p_space))])
                subs.append("Q" + r + s)
                ops.append(self.Bb[(_space(r, p_space), _space(s, p_space))])
            elif name == "f":
                a, b = idx
                sp = _space(a, p_space)
                e = self.eo if sp == "o" else self.ev
                subs.append(idx)
                ops.append(np.diag(e))
            elif name == "Y1":
                if y1_eye is not None:
                    subs.append(idx + y1_eye)
                    ops.append(np.eye(self.n1))
                else:
                    subs.append("z" + idx)
                    ops.append(Y1)
            elif name == "Y2":
                subs.append("z" + idx)
                ops.append(Y2)
            else:
                if name not in self.T:
                    self._third_order()
                subs.append(idx)
                ops.append(self.T[name])
        return subs, ops

    def _eval(self, terms, out, magnitude=False, **kw):
        """Sum of the terms; magnitude=True sums |coef| times the product of
        the operands' absolute values instead (a bound on every partial sum any
        regrouping of the same terms can form)."""
        acc = None
        for coef, spec in terms:
            subs, ops = self._operands(spec, **kw)
            c = float(eval_fraction(coef))
            if magnitude:
                c, ops = abs(c), [np.abs(op) for op in ops]
            val = c * _einsum_sliced(subs, out, ops)
            acc = val if acc is None else acc + val
        return acc

    # ------------------------------------------------------------------
    # step 2: amplitudes (Eqs. 13-14)
    # ------------------------------------------------------------------
    def _amplitudes(self):
        eo, ev = self.eo, self.ev
        D1 = ev[None, :] - eo[:, None]                                   # e_a - e_i
        D2 = (ev[None, None, :, None] + ev[None, None, None, :]
              - eo[:, None, None, None] - eo[None, :, None, None])       # e_a+e_b-e_i-e_j
        Bov = self.Bb[("o", "v")]
        ovov = _ovov(Bov)
        self.T["t"] = -ovov.transpose(0, 2, 1, 3) / D2                # (ia|jb)/(ei+ej-ea-eb)
        amp = radc_terms.AMP_TERMS
        self.T["s"] = -self._eval(amp["t1_2"], "ia") / D1
        self.T["Ds"] = D1 * self.T["s"]
        self.D1, self.D2 = D1, D2

    def _third_order(self):
        """Second-order doubles u and third-order singles w (order 3 only)."""
        if self.order < 3 or "u" in self.T:
            return
        amp = radc_terms.AMP_TERMS
        self.T["u"] = -self._eval(amp["t2_2"], "ijab") / self.D2
        self.T["Du"] = self.D2 * self.T["u"]
        self.T["w"] = -self._eval(amp["t1_3"], "ia") / self.D1

    def mp_energy(self, k):
        """k-th order correlation energy: E(2) from t, E(3) from u (closed shell)."""
        ovov = _ovov(self.Bb[("o", "v")])
        x = self.T["t"] if k == 2 else self.T["u"]
        return float(np.einsum("ijab,iajb->", x, 2 * ovov - ovov.transpose(0, 3, 2, 1)))

    # ------------------------------------------------------------------
    # step 3: the 1p-1p / 1h-1h block
    # ------------------------------------------------------------------
    def _blocks(self, blk):
        n = self.order
        lim = n - blk.count("2")
        return [(c, s) for key, lst in self.terms.items()
                if key.split("/")[0] == blk and int(key.split("/")[1]) <= lim
                for (c, s) in lst]

    def _m11(self):
        ext = "a" if self.kind == "ea" else "i"
        return self._eval(self._blocks("11"), ext + "Y", y1_eye="Y")

    # ------------------------------------------------------------------
    # Z <-> Y pair transforms
    # ------------------------------------------------------------------
    def _pair_axes(self):
        # Y2 internal layout: EA [a, b, i] (pair axes 0, 1); IP [i, j, a] (pair axes 0, 1)
        return (1, 0, 2)

    def z_to_y(self, Z2):
        return ALI * Z2 + BEI * Z2.transpose(0, 2, 1, 3)

    def y_to_z(self, Y2):
        return AL * Y2 + BE * Y2.transpose(0, 2, 1, 3)

    def unpack(self, vecs):
        """[nvec, dim] -> (Z1 [nvec, n1], Z2 [nvec, x, x, y]) in internal layout."""
        vecs = np.atleast_2d(np.asarray(vecs, dtype=np.float64))
        O, V = self.O, self.V
        Z1 = vecs[:, :self.n1]
        if self.kind == "ea":
            Z2 = vecs[:, self.n1:].reshape(-1, O, V, V).transpose(0, 2, 3, 1)   # [z,a,b,i]
        else:
            Z2 = vecs[:, self.n1:].reshape(-1, V, O, O).transpose(0, 2, 3, 1)   # [z,i,j,a]
        return np.ascontiguousarray(Z1), np.ascontiguousarray(Z2)

    def pack(self, Z1, Z2):
        nv = Z1.shape[0]
        if self.kind == "ea":
            t = Z2.transpose(0, 3, 1, 2)      # [z,i,a,b]
        else:
            t = Z2.transpose(0, 3, 1, 2)      # [z,a,i,j]
        return np.concatenate([Z1, t.reshape(nv, -1)], axis=1)

    # ------------------------------------------------------------------
    # step 4: sigma = M Z
    # ------------------------------------------------------------------
    def sigma_y(self, Y1, Y2, skip_11=False, magnitude=False):
        """Rows of M_Y Y (the non-symmetric representation of Eqs. 36-37).

        skip_11 leaves out the 1p-1p / 1h-1h product (used to time the rest
        without building M11); magnitude: see sigma_magnitude."""
        if self.kind == "ea":
            e1, e2 = "za", "zabi"
        else:
            e1, e2 = "zi", "zija"
        M11 = np.abs(self.M11) if magnitude and not skip_11 else None
        if skip_11:
            s1 = np.zeros_like(Y1)
        else:
            s1 = np.einsum("xy,zy->zx", M11 if magnitude else self.M11, Y1)
        s1 = s1 + self._eval(self._blocks("12"), e1, magnitude=magnitude, Y1=Y1, Y2=Y2)
        s2 = self._eval(self._blocks("21") + self._blocks("22"), e2, magnitude=magnitude,
                        Y1=Y1, Y2=Y2)
        return s1, s2

    def sigma(self, vecs, skip_11=False):
        """sigma = M_Z X for X [nvec, dim] (boundary layout)."""
        Z1, Z2 = self.unpack(vecs)
        Y2 = self.z_to_y(Z2)
        s1, s2 = self.sigma_y(Z1, Y2, skip_11=skip_11)
        return self.pack(s1, self.y_to_z(s2))

    def sigma_rows(self, vecs, rows):
        """Selected elements of the 2p1h (EA) / 2h1p (IP) part of sigma = M_Z X,
        each computed on its own (for systems whose whole sigma is out of reach):
        rows are (x, p, q) in the boundary layout Z2[x][p][q] (EA: (i, a, b),
        IP: (a, i, j)).  Every 21 and 22 term of the Y rows is evaluated with
        its output indices fixed, for the row (p, q, x) and its pair partner
        (q, p, x), then mapped to the Z basis (the 2x2 pair transform).
        Returns [nvec, nrows]."""
        Z1, Z2 = self.unpack(vecs)
        Y2 = self.z_to_y(Z2)
        ext = "abi" if self.kind == "ea" else "ija"
        terms = self._blocks("21") + self._blocks("22")
        out = np.zeros((Z1.shape[0], len(rows)))
        for r, (x, p, q) in enumerate(rows):
            vals = []
            for (u, w) in ((p, q), (q, p)):
                fixed = {ext[0]: u, ext[1]: w, ext[2]: x}
                acc = np.zeros(Z1.shape[0])
                for coef, spec in terms:
                    subs, ops = self._operands(spec, Y1=Z1, Y2=Y2)
                    sops = []
                    for sub, op in zip(subs, ops):
                        sl = tuple(slice(fixed[c], fixed[c] + 1) if c in fixed else slice(None)
                                   for c in sub)
                        sops.append(op[sl])
                    val = np.einsum(",".join(subs) + "->z" + ext, *sops, optimize=True)
                    acc += float(eval_fraction(coef)) * val.reshape(Z1.shape[0])
                vals.append(acc)
            out[:, r] = AL * vals[0] + BE * vals[1] if p != q else vals[0]
        return out

    def sigma_magnitude(self, vecs):
        """Scale for rounding-error bounds of sigma, element by element: the
        same sums as sigma with every coefficient, tensor, metric factor and
        vector element replaced by its absolute value, so that each element
        bounds the absolute values of the products that make up that element
        of sigma = M_Z X (and of any regrouping of those products).  Not a
        result of the method: only the scale against which a reduced-precision
        sigma is compared."""
        Z1, Z2 = self.unpack(vecs)
        Z1, Z2 = np.abs(Z1), np.abs(Z2)
        Y2 = ALI * Z2 + abs(BEI) * Z2.transpose(0, 2, 1, 3)
        s1, s2 = self.sigma_y(Z1, Y2, magnitude=True)
        s2 = AL * s2 + abs(BE) * s2.transpose(0, 2, 1, 3)
        return self.pack(s1, s2)

    def explicit(self):
        """Explicit M_Z (dim x dim) by sigma on unit vectors (small cases only)."""
        return self.sigma(np.eye(self.dim)).T

    def diag(self):
        """Exact diagonal of M_Z."""
        ext = "abi" if self.kind == "ea" else "ija"
        terms = self._blocks("22")
        d0 = self._delta_diag(terms, ext, swap=False)
        d1 = self._delta_diag(terms, ext, swap=True)
        # H = S M_Y on the pair block, then S^{-1/2} H S^{-1/2}
        d0s, d1s = d0.transpose(1, 0, 2), d1.transpose(1, 0, 2)
        H_aa = 2.0 * d0 - d1s
        H_ab = 2.0 * d1 - d0s
        H_bb = 2.0 * d0s - d1
        d2 = ALI * ALI * H_aa + 2.0 * ALI * BEI * H_ab + BEI * BEI * H_bb
        x = np.arange(d2.shape[0])
        d2[x, x, :] = d0[x, x, :]
        d1p = np.diag(self.M11).copy()
        return self.pack(d1p[None, :], d2[None])[0]

    def _delta_diag(self, terms, ext, swap):
        """M_Y[(xyz),(x'y'z')] on x'y'z' = xyz (swap: x'y'z' = yxz) for 22 terms."""
        O, V = self.O, self.V
        shape = (V, V, O) if self.kind == "ea" else (O, O, V)
        out = np.zeros(shape)
        target = (ext[1] + ext[0] + ext[2]) if swap else ext
        for coef, spec in terms:
            toks = _parse(spec)
            yidx = [idx for name, idx in toks if name == "Y2"][0]
            # unify Y2's letters with the target letters
            parent = {}

            def find(c):
                while parent.get(c, c) != c:
                    c = parent[c]
                return c
            for yl, tl in zip(yidx, target):
                ry, rt = find(yl), find(tl)
                if ry != rt:
                    # keep external letters as representatives
                    if ry in ext:
                        parent[rt] = ry
                    else:
                        parent[ry] = rt
            subs, ops = [], []
            for name, idx in toks:
                if name == "Y2":
                    continue
                s2, o2 = self._operands(name + ":" + idx)
                subs += ["".join(find(c) for c in s) for s in s2]
                ops += o2
            outl = [find(c) for c in ext]
            uniq = "".join(dict.fromkeys(outl))
            used = set("".join(subs))
            for c in uniq:
                if c not in used:     # value independent of this index
                    subs.append(c)
                    ops.append(np.ones(self.O if _space(c) == "o" else self.V))
            val = np.einsum(",".join(subs) + "->" + uniq, *ops, optimize="optimal")
            view = _diag_view(out, outl, uniq)
            view += float(eval_fraction(coef)) * val
        return out

    # ------------------------------------------------------------------
    # step 5: spectroscopic amplitudes and factors (Eqs. 16, 46-50)
    # ------------------------------------------------------------------
    def spec_amplitudes(self, vecs):
        """X_p for each vector: returns [nvec, N] (occupied first)."""
        Z1, Z2 = self.unpack(vecs)
        Y2 = self.z_to_y(Z2)
        n = self.order
        out = []
        for key, space in (("X_p_o", "o"), ("X_p_v", "v")):
            acc = None
            for k in range(n + 1):
                terms = self.terms.get(f"{key}/{k}", [])
                sel = []
                for c, s in terms:
                    has2 = "Y2:" in s
                    if (has2 and k <= n - 1) or ((not has2) and k <= n):
                        sel.append((c, s))
                if sel:
                    val = self._eval(sel, "zp", Y1=Z1, Y2=Y2, p_space=space)
                    acc = val if acc is None else acc + val
            if acc is None:
                acc = np.zeros((Z1.shape[0], self.O if space == "o" else self.V))
            out.append(acc)
        return np.concatenate(out, axis=1)

    def spec_factors(self, vecs):
        """P = 2 sum_p X_p^2 (Eq. 50) for normalised vectors in the Z basis."""
        X = self.spec_amplitudes(vecs)
        return 2.0 * np.sum(X * X, axis=1)


def _ovov(Bov):
    """(ia|jb) = sum_Q B^Q_ia B^Q_jb (Eq. 38) as one matrix product over Q."""
    Q, O, V = Bov.shape
    flat = Bov.reshape(Q, O * V)
    return (flat.T @ flat).reshape(O, V, O, V)


# Largest intermediate (elements) a single einsum step may create; bigger terms
# are evaluated slice by slice along an output index (the same sum, split over
# the values of one free index).
EINSUM_LIMIT = 2.0e8


def _einsum_sliced(subs, out, ops):
    expr = ",".join(subs) + "->" + out
    path, info = np.einsum_path(expr, *ops, optimize=("optimal", 1e30))
    biggest = 0.0
    for line in info.split("\n"):
        if line.strip().startswith("Largest intermediate"):
            biggest = float(line.split(":")[1].split()[0])
    if biggest <= EINSUM_LIMIT or not out:
        return np.einsum(expr, *ops, optimize=path)
    # split along the output index with the largest extent
    sizes = {}
    for sub, op in zip(subs, ops):
        for c, n in zip(sub, op.shape):
            sizes[c] = n
    ax = max(out, key=lambda c: sizes[c])
    n = sizes[ax]
    if n <= 1:
        return np.einsum(expr, *ops, optimize=path)
    nchunk = int(min(n, np.ceil(biggest / EINSUM_LIMIT)))
    bounds = np.linspace(0, n, nchunk + 1).astype(int)
    parts = []
    for lo, hi in zip(bounds[:-1], bounds[1:]):
        sops = []
        for sub, op in zip(subs, ops):
            if ax in sub:
                sl = [slice(None)] * op.ndim
                for k, c in enumerate(sub):
                    if c == ax:
                        sl[k] = slice(lo, hi)
                op = op[tuple(sl)]
            sops.append(op)
        parts.append(_einsum_sliced(subs, out, sops))
    return np.concatenate(parts, axis=out.index(ax))


def _diag_view(arr, letters, uniq):
    """Writable view of arr with repeated letters merged (a generalised diagonal)."""
    strides = []
    shape = []
    for u in uniq:
        st = sum(arr.strides[k] for k, c in enumerate(letters) if c == u)
        sz = [arr.shape[k] for k, c in enumerate(letters) if c == u][0]
        strides.append(st)
        shape.append(sz)
    return as_strided(arr, shape=shape, strides=strides)


def eval_fraction(s):
    if "/" in s:
        a, b = s.split("/")
        return float(a) / float(b)
    return float(s)


def eigh_lowest(M, nroots):
    w, v = np.linalg.eigh(M)
    return w[:nroots], v[:, :nroots]
