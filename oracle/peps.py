"""Oracle: amplitudes, boundary MPS, strips, local energies and log-derivatives.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``). Plain numpy in FP64 /
complex128, one configuration at a time, no blocking or fusion.

Conventions (the paper leaves them open; these are the readings taken):
  * open Lx x Ly lattice, rows x = 0..Lx-1 from the top, columns y = 0..Ly-1,
    site n = x*Ly + y;
  * site tensor T[x,y] has shape (d, Dl, Dr, Du, Dd), open-edge legs have
    dimension 1, parameters are the tensor entries in that C order, sites
    concatenated in row-major order (Sec. "Finite PEPS and Sampling");
  * a boundary MPS tensor has legs (a, k, b): left bond, physical leg, right
    bond. For the top environment E^u[i] the physical leg is the down leg of
    row i, for the bottom environment E^l[j] it is the up leg of row j.
"""
from __future__ import annotations

import math

import numpy as np


class Geometry:
    """Open square lattice with physical dimension d and virtual bond D."""

    def __init__(self, Lx: int, Ly: int, d: int, D: int):
        self.Lx, self.Ly, self.d, self.D = Lx, Ly, d, D
        self.N = Lx * Ly
        self.offset = {}
        self.block = {}
        off = 0
        for x in range(Lx):
            for y in range(Ly):
                b = int(np.prod(self.legs(x, y)))
                self.offset[(x, y)] = off
                self.block[(x, y)] = b
                off += d * b
        self.n_params = off
        self.n_compact = off // d

    def legs(self, x, y):
        D = self.D
        return (1 if y == 0 else D, 1 if y == self.Ly - 1 else D,
                1 if x == 0 else D, 1 if x == self.Lx - 1 else D)

    def compact_offset(self, x, y):
        return self.offset[(x, y)] // self.d


def site_tensors(theta, g: Geometry):
    """T[x,y] as arrays of shape (d, Dl, Dr, Du, Dd)."""
    T = {}
    for x in range(g.Lx):
        for y in range(g.Ly):
            o = g.offset[(x, y)]
            n = g.d * g.block[(x, y)]
            T[(x, y)] = np.asarray(theta[o:o + n]).reshape((g.d,) + g.legs(x, y))
    return T


def project(T, g: Geometry, s):
    """Fix every physical index to the configuration: A[x,y] = T[x,y][s_xy]."""
    return {(x, y): T[(x, y)][int(s[x * g.Ly + y])]
            for x in range(g.Lx) for y in range(g.Ly)}


# ----------------------------------------------------------------------------
# Brute force (independent of the boundary-MPS code): contract every virtual
# bond of the projected network at once (Eq. PsiS).
# ----------------------------------------------------------------------------

def _network_sublists(g: Geometry):
    """Integer bond labels for the projected network with open legs dropped."""
    lab = {}
    nxt = 0
    for x in range(g.Lx):
        for y in range(g.Ly - 1):
            lab[('h', x, y)] = nxt
            nxt += 1
    for x in range(g.Lx - 1):
        for y in range(g.Ly):
            lab[('v', x, y)] = nxt
            nxt += 1
    subs = {}
    for x in range(g.Lx):
        for y in range(g.Ly):
            s = []
            if y > 0:
                s.append(lab[('h', x, y - 1)])
            if y < g.Ly - 1:
                s.append(lab[('h', x, y)])
            if x > 0:
                s.append(lab[('v', x - 1, y)])
            if x < g.Lx - 1:
                s.append(lab[('v', x, y)])
            subs[(x, y)] = s
    return subs


def _squeeze(t):
    return t.reshape([n for n in t.shape if n != 1]) if t.ndim else t


def brute_amplitude(A, g: Geometry, skip=None, path=None):
    """Psi(S) = tTr prod A[x,y] by one einsum over all bonds (Eq. PsiS).

    With ``skip=(x, y)`` the tensor at that site is left out and the open
    legs are returned in (l, r, u, d) order: the hole tensor dPsi/dA[x,y]
    (the gradient network of Sec. "Finite PEPS and Sampling").
    """
    subs = _network_sublists(g)
    args = []
    for key in sorted(subs):
        if key == skip:
            continue
        args += [_squeeze(A[key]), subs[key]]
    if skip is None:
        out = []
    else:
        out = subs[skip]
    args.append(out)
    res = np.einsum(*args, optimize=path if path is not None else 'greedy')
    if skip is None:
        return complex(res) if np.iscomplexobj(res) else float(res)
    return np.asarray(res).reshape(g.legs(*skip))


def exact_amplitudes(theta, g: Geometry, configs):
    """Brute-force amplitude of every configuration in ``configs``."""
    T = site_tensors(theta, g)
    subs = _network_sublists(g)
    out = np.empty(len(configs), dtype=np.result_type(theta.dtype, np.float64))
    path = None
    for i, s in enumerate(configs):
        A = project(T, g, s)
        if path is None:
            args = []
            for key in sorted(subs):
                args += [_squeeze(A[key]), subs[key]]
            args.append([])
            path = np.einsum_path(*args, optimize='greedy')[0]
        out[i] = brute_amplitude(A, g, path=path)
    return out


# ----------------------------------------------------------------------------
# Boundary MPS (Sec. "On the boundary MPS method", Eq. boundary_MPS_approx)
# ----------------------------------------------------------------------------

def top_row_mps(A, g: Geometry, x: int = 0):
    """Row x read as an MPS with the down legs as physical legs (A[l,r,1,d])."""
    return [A[(x, y)][:, :, 0, :].transpose(0, 2, 1) for y in range(g.Ly)]


def bottom_row_mps(A, g: Geometry, x: int):
    """Row x read as an MPS with the up legs as physical legs (A[l,r,u,1])."""
    return [A[(x, y)][:, :, :, 0].transpose(0, 2, 1) for y in range(g.Ly)]


def absorb(mps, A, g: Geometry, x: int, from_top: bool):
    """Exact MPS x row-MPO product; the bond grows from chi to chi*D.

    From the top, the MPS physical leg joins the up legs of row x and the
    new physical leg is the down leg; from the bottom the roles swap.
    """
    out = []
    for y, E in enumerate(mps):
        a = A[(x, y)]
        if from_top:
            P = np.einsum('aub,lrud->aldbr', E, a)
        else:
            P = np.einsum('adb,lrud->alubr', E, a)
        s = P.shape
        out.append(P.reshape(s[0] * s[1], s[2], s[3] * s[4]))
    return out


def kept_count(sv, chi: int, cutoff: float = 0.0) -> int:
    """Singular values kept at one bond. Fixed chi: min(chi, len(sv)). With a
    maximal truncated weight (Sec. "On the boundary MPS method": D_c chosen
    dynamically, cutoff 1e-4 in the paper's runs) the smallest r <= chi whose
    discarded weight sum_{k>=r} sv_k^2 / sum_k sv_k^2 is at most the cutoff;
    chi itself when even chi values discard more."""
    sv = np.asarray(sv, dtype=np.float64)
    r = min(chi, len(sv))
    if cutoff <= 0.0 or r <= 1:
        return r
    w = sv ** 2
    lim = cutoff * w.sum()
    tail = w[r:].sum()
    if tail > lim:
        return r
    for j in range(r - 1, 0, -1):
        t2 = tail + w[j]
        if t2 > lim:
            return j + 1
        tail = t2
    return 1


def compress_canonical(mps, chi: int, cutoff: float = 0.0):
    """Truncate every bond to chi: left-to-right QR sweep, then a
    right-to-left SVD sweep keeping the chi largest singular values (with a
    cutoff > 0: the fewest that keep the discarded weight within it, see
    ``kept_count``).

    This is the canonical way of truncating an MPS-MPO product; it yields the
    same truncated state as the density-matrix algorithm the paper uses
    (``compress_density_matrix``).
    """
    n = len(mps)
    Q = [None] * n
    M = mps[0]
    for y in range(n - 1):
        bl, k, br = M.shape
        q, r = np.linalg.qr(M.reshape(bl * k, br))
        Q[y] = q.reshape(bl, k, q.shape[1])
        M = np.einsum('ij,jkb->ikb', r, mps[y + 1])
    Q[n - 1] = M
    out = [None] * n
    X = None
    for y in range(n - 1, 0, -1):
        C = Q[y] if X is None else np.einsum('akb,bc->akc', Q[y], X)
        bl, k, br = C.shape
        u, sv, vh = np.linalg.svd(C.reshape(bl, k * br), full_matrices=False)
        r = kept_count(sv, chi, cutoff)
        out[y] = vh[:r].reshape(r, k, br)
        X = u[:, :r] * sv[:r]
    out[0] = np.einsum('akb,bc->akc', Q[0], X) if n > 1 else Q[0]
    return out


def compress_density_matrix(mps, chi: int, cutoff: float = 0.0):
    """The density-matrix MPS-MPO truncation (Sec. "On the boundary MPS
    method"): left Gram environments of the untruncated product, then from
    the right the reduced density matrix of each site is diagonalised and
    its chi dominant eigenvectors become the new right-isometric tensor.
    The eigenvalues are the squared singular values of the canonical centre
    matrix, so a maximal truncated weight (``kept_count``) applies to their
    square roots.
    """
    n = len(mps)
    G = [None] * n
    G[0] = np.ones((1, 1))
    for y in range(n - 1):
        P = mps[y]
        G[y + 1] = np.einsum('ab,akc,bkd->cd', G[y], P.conj(), P, optimize='greedy')
    out = [None] * n
    W = np.ones((1, 1))
    for y in range(n - 1, 0, -1):
        Z = np.einsum('akb,bc->akc', mps[y], W)
        bl, k, r0 = Z.shape
        Zm = Z.reshape(bl, k * r0)
        rho = Zm.T @ G[y].T @ Zm.conj()
        rho = 0.5 * (rho + rho.conj().T)
        w, V = np.linalg.eigh(rho)
        order = np.argsort(w)[::-1]
        sv = np.sqrt(np.clip(w[order], 0.0, None))[:min(bl, k * r0)]
        r = kept_count(sv, chi, cutoff)
        order = order[:r]
        Bt = V[:, order].T.reshape(r, k, r0)
        out[y] = Bt
        W = np.einsum('akc,jkc->aj', Z, Bt.conj())
    out[0] = np.einsum('akb,bc->akc', mps[0], W)
    return out


def normalize(mps):
    """Divide each tensor by its largest modulus and return the sum of the
    logarithms of the divisors (Sec. "On Numerical Stability")."""
    logf = 0.0
    out = []
    for t in mps:
        f = float(np.max(np.abs(t)))
        if f == 0.0:
            out.append(t)
            logf += -math.inf
            continue
        out.append(t / f)
        logf += math.log(f)
    return out, logf


def _compressor(method: str, cutoff: float):
    if method == 'canonical':
        return lambda m, chi: compress_canonical(m, chi, cutoff)
    return lambda m, chi: compress_density_matrix(m, chi, cutoff)


def top_environments(A, g: Geometry, chi: int, method: str = 'canonical', cutoff: float = 0.0):
    """E^u[i] for i = 0..Lx-2 and their log scales: E^u[0] is row 0, each
    further one absorbs a row, truncates to chi and renormalises."""
    comp = _compressor(method, cutoff)
    U, fU = {}, {}
    mps, f = normalize(top_row_mps(A, g, 0))
    U[0], fU[0] = mps, f
    for x in range(1, g.Lx - 1):
        mps = comp(absorb(U[x - 1], A, g, x, True), chi)
        mps, df = normalize(mps)
        U[x], fU[x] = mps, fU[x - 1] + df
    return U, fU


def bottom_environments(A, g: Geometry, chi: int, method: str = 'canonical',
                        cutoff: float = 0.0):
    """E^l[j] for j = Lx-1..1 (mirror image of ``top_environments``)."""
    comp = _compressor(method, cutoff)
    B, fB = {}, {}
    L = g.Lx - 1
    mps, f = normalize(bottom_row_mps(A, g, L))
    B[L], fB[L] = mps, f
    for x in range(L - 1, 0, -1):
        mps = comp(absorb(B[x + 1], A, g, x, False), chi)
        mps, df = normalize(mps)
        B[x], fB[x] = mps, fB[x + 1] + df
    return B, fB


def overlap(top, bottom):
    """Contract two boundary MPS over their physical legs (E^u[i] . E^l[i+1])."""
    L = np.ones((1, 1), dtype=np.result_type(top[0], bottom[0]))
    for a, b in zip(top, bottom):
        L = np.einsum('ac,akb,ckd->bd', L, a, b, optimize='greedy')
    return L[0, 0]


def clog(z) -> complex:
    """Principal complex logarithm (log|z| + i arg z)."""
    z = complex(z)
    if z == 0:
        return complex(-math.inf, 0.0)
    return complex(math.log(abs(z)), math.atan2(z.imag, z.real))


def log_amplitude_at(U, fU, B, fB, i: int) -> complex:
    """ln Psi(S)_i = ln(E^u[i] . E^l[i+1]) plus both log scales."""
    return clog(overlap(U[i], B[i + 1])) + fU[i] + fB[i + 1]


def amplitude_row_index(g: Geometry) -> int:
    """The cut i* = floor(Lx/2) - 1 at which ln Psi is reported (the paper's
    example uses i = 5 of L = 10, counted from 1)."""
    return g.Lx // 2 - 1


# ----------------------------------------------------------------------------
# Strips: one row (or two rows) between a top and a bottom environment, with
# left and right partial contractions (Sec. "On reusing environments").
# ----------------------------------------------------------------------------

def _c(spec, a, b):
    """One pairwise contraction (einsum with a BLAS-backed path)."""
    return np.einsum(spec, a, b, optimize=True)


def _trivial_mps(Ly, dtype):
    return [np.ones((1, 1, 1), dtype=dtype) for _ in range(Ly)]


class Strip1:
    """Row x between E^u[x-1] and E^l[x+1]; Lf[y+1] holds sites 0..y."""

    def __init__(self, Up, row, Bt):
        self.Up, self.row, self.Bt = Up, row, Bt
        n = len(row)
        dt = np.result_type(Up[0], row[0], Bt[0])
        self.Lf = [None] * (n + 1)
        self.Rt = [None] * (n + 1)
        self.Lf[0] = np.ones((1, 1, 1), dtype=dt)
        for y in range(n):
            self.Lf[y + 1] = self.step_left(self.Lf[y], y, row[y])
        self.Rt[n] = np.ones((1, 1, 1), dtype=dt)
        for y in range(n - 1, -1, -1):
            self.Rt[y] = self.step_right(self.Rt[y + 1], y, row[y])
        self.value = np.einsum('amc,amc->', self.Lf[n], self.Rt[n])

    def step_left(self, L, y, a):
        X = _c('amc,aub->mcub', L, self.Up[y])
        X = _c('mcub,mrud->cbrd', X, a)
        return _c('cbrd,cde->bre', X, self.Bt[y])

    def step_right(self, R, y, a):
        X = _c('bre,aub->reau', R, self.Up[y])
        X = _c('reau,mrud->eamd', X, a)
        return _c('eamd,cde->amc', X, self.Bt[y])

    def window(self, y0, tensors):
        """Strip value with sites y0.. replaced by ``tensors``."""
        L = self.Lf[y0]
        for j, a in enumerate(tensors):
            L = self.step_left(L, y0 + j, a)
        return np.einsum('amc,amc->', L, self.Rt[y0 + len(tensors)])

    def hole(self, y):
        """d(strip value)/d(row tensor y), legs (l, r, u, d)."""
        X = _c('amc,aub->mcub', self.Lf[y], self.Up[y])
        X = _c('mcub,cde->mubde', X, self.Bt[y])
        return _c('mubde,bre->mrud', X, self.Rt[y + 1])


class Strip2:
    """Rows x, x+1 between E^u[x-1] and E^l[x+2]."""

    def __init__(self, Up, row1, row2, Bt):
        self.Up, self.r1, self.r2, self.Bt = Up, row1, row2, Bt
        n = len(row1)
        dt = np.result_type(Up[0], row1[0], Bt[0])
        self.Lf = [None] * (n + 1)
        self.Rt = [None] * (n + 1)
        self.Lf[0] = np.ones((1, 1, 1, 1), dtype=dt)
        for y in range(n):
            self.Lf[y + 1] = self.step_left(self.Lf[y], y, row1[y], row2[y])
        self.Rt[n] = np.ones((1, 1, 1, 1), dtype=dt)
        for y in range(n - 1, -1, -1):
            self.Rt[y] = self.step_right(self.Rt[y + 1], y, row1[y], row2[y])
        self.value = np.einsum('amnc,amnc->', self.Lf[n], self.Rt[n])

    def step_left(self, L, y, a1, a2):
        X = _c('amnc,aub->mncub', L, self.Up[y])
        X = _c('mncub,mrut->ncbrt', X, a1)
        X = _c('ncbrt,nstd->cbrsd', X, a2)
        return _c('cbrsd,cde->brse', X, self.Bt[y])

    def step_right(self, R, y, a1, a2):
        X = _c('brse,cde->brscd', R, self.Bt[y])
        X = _c('brscd,nstd->brcnt', X, a2)
        X = _c('brcnt,mrut->bcnmu', X, a1)
        return _c('bcnmu,aub->amnc', X, self.Up[y])

    def window(self, y0, cols):
        L = self.Lf[y0]
        for j, (a1, a2) in enumerate(cols):
            L = self.step_left(L, y0 + j, a1, a2)
        return np.einsum('amnc,amnc->', L, self.Rt[y0 + len(cols)])


class SampleContraction:
    """Everything the estimators need for one configuration: the cached
    environments, the amplitude at the middle cut and lazily built strips."""

    def __init__(self, T, g: Geometry, s, chi: int, method: str = 'canonical',
                 cutoff: float = 0.0):
        self.T, self.g, self.s, self.chi = T, g, np.asarray(s), chi
        self.A = project(T, g, s)
        self.U, self.fU = top_environments(self.A, g, chi, method, cutoff)
        self.B, self.fB = bottom_environments(self.A, g, chi, method, cutoff)
        self.istar = amplitude_row_index(g)
        self.logpsi = log_amplitude_at(self.U, self.fU, self.B, self.fB, self.istar)
        self._s1 = {}
        self._s2 = {}

    def _up(self, x):
        dt = self.A[(0, 0)].dtype
        return self.U[x - 1] if x > 0 else _trivial_mps(self.g.Ly, dt)

    def _down(self, x):
        dt = self.A[(0, 0)].dtype
        return self.B[x + 1] if x < self.g.Lx - 1 else _trivial_mps(self.g.Ly, dt)

    def row(self, x):
        return [self.A[(x, y)] for y in range(self.g.Ly)]

    def strip1(self, x) -> Strip1:
        if x not in self._s1:
            self._s1[x] = Strip1(self._up(x), self.row(x), self._down(x))
        return self._s1[x]

    def strip2(self, x) -> Strip2:
        if x not in self._s2:
            self._s2[x] = Strip2(self._up(x), self.row(x), self.row(x + 1),
                                 self._down(x + 1))
        return self._s2[x]

    def ratio(self, changes):
        """Psi(S')/Psi(S) for S' = S with ``changes`` = {site: new value},
        evaluated inside the strip that holds the changed sites and reusing
        its environments outside the support (Sec. "On reusing environments").
        The two amplitudes of the ratio come from the same strip."""
        g = self.g
        xs = sorted({n // g.Ly for n in changes})
        ys = sorted({n % g.Ly for n in changes})
        y0, y1 = ys[0], ys[-1]
        if len(xs) == 1:
            x = xs[0]
            st = self.strip1(x)
            ts = []
            for y in range(y0, y1 + 1):
                n = x * g.Ly + y
                p = changes.get(n, int(self.s[n]))
                ts.append(self.T[(x, y)][p])
            num = st.window(y0, ts)
            den = st.value
        elif len(xs) == 2 and xs[1] == xs[0] + 1:
            x = xs[0]
            st = self.strip2(x)
            cols = []
            for y in range(y0, y1 + 1):
                n1, n2 = x * g.Ly + y, (x + 1) * g.Ly + y
                p1 = changes.get(n1, int(self.s[n1]))
                p2 = changes.get(n2, int(self.s[n2]))
                cols.append((self.T[(x, y)][p1], self.T[(x + 1, y)][p2]))
            num = st.window(y0, cols)
            den = st.value
        else:
            raise ValueError('term spans more than two adjacent rows')
        return num / den

    def local_energy(self, ham) -> complex:
        """E_loc(S) = sum_t sum_S' <S|h_t|S'> Psi(S')/Psi(S) (Eq. local_obs,
        matrix element read as <S|H|S'>); diagonal long-range pairs need no
        amplitude (Sec. "On reusing environments")."""
        e = 0.0 + 0.0j
        s = self.s
        for sites, h in ham.terms:
            k = len(sites)
            c = 0
            for n in sites:
                c = 2 * c + int(s[n])
            row = h[c]
            for c2 in np.nonzero(row)[0]:
                c2 = int(c2)
                if c2 == c:
                    e += row[c]
                    continue
                changes = {}
                for j, n in enumerate(sites):
                    b = (c2 >> (k - 1 - j)) & 1
                    if b != int(s[n]):
                        changes[n] = b
                e += row[c2] * self.ratio(changes)
        e += ham.diagonal(s)
        return complex(e)

    def logderiv_compact(self):
        """O_k = d ln Psi_row(x) / d theta_k for the parameters of every site
        (x, y) with p = s_xy: the hole network of the row strip divided by
        the strip amplitude (Sec. "Finite PEPS and Sampling", Eq. tdvp; the
        boundary-MPS gradients of Sec. "On the boundary MPS method"). The
        entries with p != s_xy are zero and are not stored."""
        g = self.g
        out = np.zeros(g.n_compact, dtype=np.result_type(self.A[(0, 0)], np.float64))
        for x in range(g.Lx):
            st = self.strip1(x)
            for y in range(g.Ly):
                h = st.hole(y) / st.value
                o = g.compact_offset(x, y)
                out[o:o + h.size] = h.ravel()
        return out


def local_energy_strict(theta, g: Geometry, configs, chi: int, ham, method='canonical',
                        cutoff: float = 0.0):
    """E_loc with every amplitude taken from the full boundary-MPS contraction
    at the one cut i* (Sec. "On Variational Upper Bound"):
    E_loc(S) = sum_S' <S|H|S'> Psi(S')_i* / Psi(S)_i*. Averaged over
    p(S) ~ |Psi(S)_i*|^2 this is the energy of the single vector
    S -> Psi(S)_i*, so it cannot fall below the ground-state energy; the strip
    ratios of ``SampleContraction.local_energy`` do not have that property at
    a truncating chi."""
    T = site_tensors(theta, g)
    out = np.empty(len(configs), dtype=np.complex128)
    for idx, s in enumerate(configs):
        s = np.asarray(s)
        l0 = SampleContraction(T, g, s, chi, method, cutoff).logpsi
        e = 0.0 + 0.0j
        for sites, h in ham.terms:
            k = len(sites)
            c = 0
            for n in sites:
                c = 2 * c + int(s[n])
            row = h[c]
            for c2 in np.nonzero(row)[0]:
                c2 = int(c2)
                if c2 == c:
                    e += row[c]
                    continue
                s2 = s.copy()
                for j, n in enumerate(sites):
                    s2[n] = (c2 >> (k - 1 - j)) & 1
                l1 = SampleContraction(T, g, s2, chi, method, cutoff).logpsi
                e += row[c2] * np.exp(l1 - l0)
        e += ham.diagonal(s)
        out[idx] = e
    return out


def expand_compact(Oc, g: Geometry, s):
    """Full O row (N_p entries) from the compact one: zeros where p != s_xy."""
    out = np.zeros(g.n_params, dtype=Oc.dtype)
    for x in range(g.Lx):
        for y in range(g.Ly):
            b = g.block[(x, y)]
            o = g.offset[(x, y)] + int(s[x * g.Ly + y]) * b
            c = g.compact_offset(x, y)
            out[o:o + b] = Oc[c:c + b]
    return out


def evaluate(theta, g: Geometry, configs, chi: int, ham=None, want_O=False,
             method='canonical', cutoff: float = 0.0):
    """ln Psi, E_loc and compact O for a batch, one configuration at a time."""
    T = site_tensors(theta, g)
    n = len(configs)
    logpsi = np.empty(n, dtype=np.complex128)
    eloc = np.empty(n, dtype=np.complex128) if ham is not None else None
    O = None
    for i, s in enumerate(configs):
        sc = SampleContraction(T, g, s, chi, method, cutoff)
        logpsi[i] = sc.logpsi
        if ham is not None:
            eloc[i] = sc.local_energy(ham)
        if want_O:
            o = sc.logderiv_compact()
            if O is None:
                O = np.empty((n, o.size), dtype=o.dtype)
            O[i] = o
    return logpsi, eloc, O
