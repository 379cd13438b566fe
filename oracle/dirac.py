"""The QCD+QED O(a)-improved Wilson-Dirac operator, written from its definition.

TEST INFRASTRUCTURE ONLY (see the package docstring).

What the paper fixes (arXiv:2502.02490):
  * Sec. 2: spinor index order (x, alpha, a), colour fastest; the clover term is two
    Hermitian 6x6 blocks per site, one per chirality.
  * Sec. 4.1.3: a block is stored as 36 reals: 6 diagonal entries, then 15
    (re, im) pairs of the strictly upper triangle in row-major order.
  * Sec. 4.1.4: gauge links are 3x3 row-major; here four forward links per site.
  * Sec. 4.3: the QCD+QED link is exp(i q A_mu(x)) U_mu(x), a U(3) matrix, and the
    clover term is an SU(3) Sheikholeslami-Wohlert term plus a U(1) one with its
    own coefficient c_sw^U(1); the sum stays site- and chirality-diagonal and Hermitian.

Readings where the paper is silent (each one is listed with the library's):
  R1 gamma matrices: Euclidean, Hermitian, chiral basis,
       gamma_0 = [[0, -1], [-1, 0]],  gamma_k = [[0, -i sigma_k], [i sigma_k, 0]],
       gamma_5 = gamma_0 gamma_1 gamma_2 gamma_3 = diag(1, 1, -1, -1);
     sigma_{mu nu} = (i/2) [gamma_mu, gamma_nu].  The chiral basis is what makes the
     clover block-diagonal with an upper (+) and lower (-) block.
  R2 operator, m0 normalisation (m0 = 1/(2 kappa) - 4):
       D psi(x) = (4 + m0) psi(x) + C(x) psi(x)
                  - 1/2 sum_mu [ V_mu(x) b+_mu(x) (1 - gamma_mu) psi(x + mu)
                               + V_mu(x - mu)^dag b-_mu(x) (1 + gamma_mu) psi(x - mu) ],
       b+_mu(x) = exp(i phi_mu) if x_mu = L_mu - 1 else 1,
       b-_mu(x) = exp(-i phi_mu) if x_mu = 0 else 1.
  R3 the integer charge qhat multiplies the angle: V_mu(x) = exp(i qhat theta_mu(x)) U_mu(x).
  R4 clover term, summed over all ordered pairs mu != nu:
       C(x) = c_sw (i/4) sigma_{mu nu} F_{mu nu}(x)
            + c_sw^QED qhat (i/4) sigma_{mu nu} F^U(1)_{mu nu}(x) (x) 1_colour,
       F = (Q - Q^dag) / 8 with Q the sum of the four plaquette leaves at x, built
       from U alone (SU(3)) or from z = exp(i theta) alone (U(1)); no traceless
       projection; the charge enters the U(1) term linearly; boundary phases do
       not enter C.
  R5 even-odd form: D = [[A_ee, D_eo], [D_oe, A_oo]],
       D-hat = A_ee - D_eo A_oo^-1 D_oe on the even sites.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import geometry as geo

# ---------------------------------------------------------------- gamma matrices (R1)
_I2 = np.eye(2, dtype=np.complex128)
_Z2 = np.zeros((2, 2), dtype=np.complex128)
PAULI = [
    np.array([[0, 1], [1, 0]], dtype=np.complex128),
    np.array([[0, -1j], [1j, 0]], dtype=np.complex128),
    np.array([[1, 0], [0, -1]], dtype=np.complex128),
]


def _blocks(a, b, c, d):
    return np.block([[a, b], [c, d]])


GAMMA = [_blocks(_Z2, -_I2, -_I2, _Z2)] + [_blocks(_Z2, -1j * s, 1j * s, _Z2) for s in PAULI]
GAMMA5 = GAMMA[0] @ GAMMA[1] @ GAMMA[2] @ GAMMA[3]
ONE4 = np.eye(4, dtype=np.complex128)
SIGMA = [[0.5j * (GAMMA[m] @ GAMMA[n] - GAMMA[n] @ GAMMA[m]) for n in range(4)] for m in range(4)]


# ---------------------------------------------------------------- fields
@dataclass
class Params:
    """Operator parameters: extents (L0 = time, L1, L2, L3), kappa, c_sw, c_sw^QED, qhat, phases phi_mu."""

    dims: tuple
    kappa: float
    csw: float
    csw_qed: float
    qhat: int
    bc_phase: tuple = (np.pi, 0.0, 0.0, 0.0)
    cstar: int = 0  # C* boundary conditions in directions 1 .. cstar (geometry.shift)

    @property
    def m0(self) -> float:
        return 1.0 / (2.0 * self.kappa) - 4.0


@dataclass
class Fields:
    """Gauge background: U[site, mu] in SU(3) (3x3, row-major) and theta[site, mu] (U(1) angle), LEX order."""

    U: np.ndarray
    theta: np.ndarray
    p: Params
    _clover: dict = field(default_factory=dict, repr=False)

    def __post_init__(self):
        geo.check_dims(self.p.dims, self.p.cstar)
        V = geo.volume(self.p.dims)
        assert self.U.shape == (V, 4, 3, 3) and self.theta.shape == (V, 4)
        # R3 / Sec. 4.3: the U(3) link exp(i qhat theta) U
        self.Vlink = np.exp(1j * self.p.qhat * self.theta)[:, :, None, None] * self.U

    @property
    def V(self) -> int:
        return geo.volume(self.p.dims)

    def clover(self, sites=None) -> np.ndarray:
        """A(x) = (4 + m0) 1 + C(x) as explicit 12x12 matrices, cached for the full lattice."""
        if sites is None:
            if "A" not in self._clover:
                self._clover["A"] = clover_matrix(self, np.arange(self.V))
            return self._clover["A"]
        if "A" in self._clover:
            return self._clover["A"][sites]
        return clover_matrix(self, np.asarray(sites))

    def clover_inv(self, sites=None) -> np.ndarray:
        if sites is None:
            if "Ainv" not in self._clover:
                self._clover["Ainv"] = np.linalg.inv(self.clover())
            return self._clover["Ainv"]
        if "Ainv" in self._clover:
            return self._clover["Ainv"][sites]
        return np.linalg.inv(self.clover(sites))


# ---------------------------------------------------------------- hopping term (R2)
def _spin(mat, psi):
    """Apply a 4x4 spin matrix to psi[n, spin, colour]."""
    return np.einsum("st,ntc->nsc", mat, psi)


def hop(f: Fields, psi: np.ndarray, sites=None) -> np.ndarray:
    """H psi at `sites` (all sites if None), psi a full LEX field [V, 4, 3]:
    H psi(x) = sum_mu [ V_mu(x) b+ (1 - gamma_mu) psi(x+mu) + V_mu(x-mu)^dag b- (1 + gamma_mu) psi(x-mu) ].
    D = A - H / 2.
    """
    L = f.p.dims
    sites = np.arange(f.V) if sites is None else np.asarray(sites, dtype=np.int64)
    x = geo.coords(sites, L)
    out = np.zeros((len(sites), 4, 3), dtype=np.complex128)
    for mu in range(4):
        fwd = geo.shift(sites, L, mu, +1, f.p.cstar)
        bwd = geo.shift(sites, L, mu, -1, f.p.cstar)
        phi = f.p.bc_phase[mu]
        bplus = np.where(x[:, mu] == L[mu] - 1, np.exp(1j * phi), 1.0)
        bminus = np.where(x[:, mu] == 0, np.exp(-1j * phi), 1.0)
        t = _spin(ONE4 - GAMMA[mu], psi[fwd])
        out += bplus[:, None, None] * np.einsum("nab,nsb->nsa", f.Vlink[sites, mu], t)
        t = _spin(ONE4 + GAMMA[mu], psi[bwd])
        Vdag = np.conj(np.swapaxes(f.Vlink[bwd, mu], -1, -2))
        out += bminus[:, None, None] * np.einsum("nab,nsb->nsa", Vdag, t)
    return out


# ---------------------------------------------------------------- clover term (R4)
def _dag(m):
    return np.conj(np.swapaxes(m, -1, -2))


def leaves(W: np.ndarray, L, sites: np.ndarray, mu: int, nu: int, cstar: int = 0) -> np.ndarray:
    """Q_{mu nu}(x): sum of the four plaquettes in the (mu, nu) plane that start and end at x.
    W[site, mu] are N x N link matrices (N = 3 for SU(3), N = 1 for U(1))."""
    s = lambda lam, d, k: geo.shift(lam, L, d, k, cstar)  # noqa: E731
    x = sites
    xpm, xpn = s(x, mu, +1), s(x, nu, +1)
    xmm, xmn = s(x, mu, -1), s(x, nu, -1)
    xmm_pn = s(xmm, nu, +1)
    xmm_mn = s(xmm, nu, -1)
    xpm_mn = s(xpm, nu, -1)
    Wm, Wn = W[:, mu], W[:, nu]
    q = Wm[x] @ Wn[xpm] @ _dag(Wm[xpn]) @ _dag(Wn[x])
    q = q + Wn[x] @ _dag(Wm[xmm_pn]) @ _dag(Wn[xmm]) @ Wm[xmm]
    q = q + _dag(Wm[xmm]) @ _dag(Wn[xmm_mn]) @ Wm[xmm_mn] @ Wn[xmn]
    q = q + _dag(Wn[xmn]) @ Wm[xmn] @ Wn[xpm_mn] @ _dag(Wm[x])
    return q


def field_strength(W: np.ndarray, L, sites, mu: int, nu: int, cstar: int = 0) -> np.ndarray:
    """F_{mu nu}(x) = (Q_{mu nu} - Q_{mu nu}^dag) / 8 (no traceless projection, reading R4)."""
    q = leaves(W, L, np.asarray(sites, dtype=np.int64), mu, nu, cstar)
    return (q - _dag(q)) / 8.0


def clover_matrix(f: Fields, sites) -> np.ndarray:
    """A(x) = (4 + m0) 1_12 + C(x) at `sites`, as [n, 12, 12] with row index 3 * spin + colour."""
    L = f.p.dims
    sites = np.asarray(sites, dtype=np.int64)
    n = len(sites)
    A = np.zeros((n, 12, 12), dtype=np.complex128)
    A += (4.0 + f.p.m0) * np.eye(12)
    z = np.exp(1j * f.theta)[:, :, None, None]  # U(1) links as 1x1 matrices, charge not included (R4)
    one3 = np.eye(3)
    for mu in range(4):
        for nu in range(4):
            if mu == nu:
                continue
            F = field_strength(f.U, L, sites, mu, nu, f.p.cstar)  # [n, 3, 3]
            A += f.p.csw * 0.25j * np.einsum("st,nab->nsatb", SIGMA[mu][nu], F).reshape(n, 12, 12)
            Fq = field_strength(z, L, sites, mu, nu, f.p.cstar)[:, 0, 0]  # [n]
            A += (f.p.csw_qed * f.p.qhat * 0.25j) * np.einsum(
                "st,n,ab->nsatb", SIGMA[mu][nu], Fq, one3).reshape(n, 12, 12)
    return A


# ---------------------------------------------------------------- the operator
def apply_D(f: Fields, psi: np.ndarray, sites=None) -> np.ndarray:
    """D psi = A psi - H psi / 2 at `sites` (all sites if None)."""
    sites = np.arange(f.V) if sites is None else np.asarray(sites, dtype=np.int64)
    A = f.clover(sites)
    return np.einsum("nij,nj->ni", A, psi[sites].reshape(-1, 12)).reshape(-1, 4, 3) - 0.5 * hop(f, psi, sites)


def apply_Ddag(f: Fields, psi: np.ndarray) -> np.ndarray:
    """D^dag psi from the definition (Hermitian conjugate of every term), not from gamma_5-hermiticity."""
    # D = A - H/2 with A Hermitian; H^dag psi(x) = sum_mu [ V_mu(x) b+ (1 + gamma_mu) psi(x+mu)
    #                                              + V_mu(x-mu)^dag b- (1 - gamma_mu) psi(x-mu) ]
    L = f.p.dims
    sites = np.arange(f.V)
    x = geo.coords(sites, L)
    out = np.zeros_like(psi)
    for mu in range(4):
        fwd = geo.shift(sites, L, mu, +1, f.p.cstar)
        bwd = geo.shift(sites, L, mu, -1, f.p.cstar)
        phi = f.p.bc_phase[mu]
        bplus = np.where(x[:, mu] == L[mu] - 1, np.exp(1j * phi), 1.0)
        bminus = np.where(x[:, mu] == 0, np.exp(-1j * phi), 1.0)
        t = _spin(ONE4 + GAMMA[mu], psi[fwd])
        out += bplus[:, None, None] * np.einsum("nab,nsb->nsa", f.Vlink[sites, mu], t)
        t = _spin(ONE4 - GAMMA[mu], psi[bwd])
        out += bminus[:, None, None] * np.einsum("nab,nsb->nsa", _dag(f.Vlink[bwd, mu]), t)
    A = f.clover()
    return np.einsum("nji,nj->ni", np.conj(A), psi.reshape(-1, 12)).reshape(-1, 4, 3) - 0.5 * out


# ---------------------------------------------------------------- even-odd form (R5)
def even_odd(f: Fields):
    return geo.sites_of_parity(f.p.dims, 0), geo.sites_of_parity(f.p.dims, 1)


def _embed(f: Fields, sites, vals):
    full = np.zeros((f.V, 4, 3), dtype=np.complex128)
    full[sites] = vals
    return full


def apply_Doe(f: Fields, psi_e: np.ndarray) -> np.ndarray:
    """D_oe psi_e = -H_oe psi_e / 2: even-site input [Vh, 4, 3] (EO order) -> odd-site output."""
    ev, od = even_odd(f)
    return -0.5 * hop(f, _embed(f, ev, psi_e), od)


def apply_Deo(f: Fields, psi_o: np.ndarray) -> np.ndarray:
    """D_eo psi_o = -H_eo psi_o / 2: odd-site input -> even-site output."""
    ev, od = even_odd(f)
    return -0.5 * hop(f, _embed(f, od, psi_o), ev)


def apply_clover(f: Fields, psi_p: np.ndarray, parity: int, inverse: bool = False) -> np.ndarray:
    """A_pp psi_p or A_pp^-1 psi_p on the sites of one parity."""
    sites = geo.sites_of_parity(f.p.dims, parity)
    M = f.clover_inv(sites) if inverse else f.clover(sites)
    return np.einsum("nij,nj->ni", M, psi_p.reshape(-1, 12)).reshape(-1, 4, 3)


def apply_schur(f: Fields, psi_e: np.ndarray) -> np.ndarray:
    """D-hat psi_e = A_ee psi_e - D_eo A_oo^-1 D_oe psi_e (R5)."""
    t = apply_clover(f, apply_Doe(f, psi_e), 1, inverse=True)
    return apply_clover(f, psi_e, 0) - apply_Deo(f, t)


def apply_schur_dag(f: Fields, psi_e: np.ndarray) -> np.ndarray:
    """D-hat^dag = A_ee - (D^dag)_eo A_oo^-1 (D^dag)_oe, with the off-diagonal blocks taken from the
    full D^dag of `apply_Ddag` (A maps each parity to itself, so restricting D^dag of a field that
    lives on one parity to the other parity isolates an off-diagonal block)."""
    ev, od = even_odd(f)
    t = apply_Ddag(f, _embed(f, ev, psi_e))[od]
    t = apply_clover(f, t, 1, inverse=True)
    return apply_clover(f, psi_e, 0) - apply_Ddag(f, _embed(f, od, t))[ev]


def schur_at(f: Fields, psi_e: np.ndarray, out_sites) -> np.ndarray:
    """D-hat psi_e at a subset of even sites (LEX indices `out_sites`), computed site by site
    from the definition; used to check full-size results on sampled outputs."""
    L = f.p.dims
    ev, _ = even_odd(f)
    out_sites = np.asarray(out_sites, dtype=np.int64)
    full_e = _embed(f, ev, psi_e)
    nb = np.unique(np.concatenate([geo.shift(out_sites, L, mu, s, f.p.cstar) for mu in range(4) for s in (1, -1)]))
    t = -0.5 * hop(f, full_e, nb)
    t = np.einsum("nij,nj->ni", f.clover_inv(nb), t.reshape(-1, 12)).reshape(-1, 4, 3)
    full_t = np.zeros((f.V, 4, 3), dtype=np.complex128)
    full_t[nb] = t
    y = np.einsum("nij,nj->ni", f.clover(out_sites), full_e[out_sites].reshape(-1, 12)).reshape(-1, 4, 3)
    return y + 0.5 * hop(f, full_t, out_sites)


# ---------------------------------------------------------------- clover packing (Sec. 4.1.3)
_UPPER = [(i, j) for i in range(6) for j in range(i + 1, 6)]


def pack_clover(A: np.ndarray) -> np.ndarray:
    """[n, 12, 12] -> [n, 2, 36]: per chirality block (spins {0,1} then {2,3}), 6 diagonal reals,
    then (re, im) of the 15 strictly-upper entries in row-major order."""
    n = A.shape[0]
    out = np.zeros((n, 2, 36))
    for c in range(2):
        B = A[:, 6 * c:6 * c + 6, 6 * c:6 * c + 6]
        out[:, c, :6] = np.real(np.diagonal(B, axis1=1, axis2=2))
        for k, (i, j) in enumerate(_UPPER):
            out[:, c, 6 + 2 * k] = B[:, i, j].real
            out[:, c, 7 + 2 * k] = B[:, i, j].imag
    return out


def unpack_clover(P: np.ndarray) -> np.ndarray:
    """[n, 2, 36] -> Hermitian chirality-block-diagonal [n, 12, 12]."""
    n = P.shape[0]
    A = np.zeros((n, 12, 12), dtype=np.complex128)
    for c in range(2):
        o = 6 * c
        for i in range(6):
            A[:, o + i, o + i] = P[:, c, i]
        for k, (i, j) in enumerate(_UPPER):
            v = P[:, c, 6 + 2 * k] + 1j * P[:, c, 7 + 2 * k]
            A[:, o + i, o + j] = v
            A[:, o + j, o + i] = np.conj(v)
    return A


def singular_blocks(A: np.ndarray, rel: float = 1e-14) -> np.ndarray:
    """Reading of the singular-block rule: a 6x6 block is singular when an LU pivot (partial
    pivoting) has modulus below rel * max|A_block|.  Returns a bool [n, 2] mask."""
    import warnings

    import scipy.linalg as sla

    n = A.shape[0]
    bad = np.zeros((n, 2), dtype=bool)
    for s in range(n):
        for c in range(2):
            B = A[s, 6 * c:6 * c + 6, 6 * c:6 * c + 6]
            with warnings.catch_warnings():
                warnings.simplefilter("ignore")
                lu, _ = sla.lu_factor(B, check_finite=False)
            bad[s, c] = np.abs(np.diag(lu)).min() < rel * np.abs(B).max()
    return bad


# ---------------------------------------------------------------- dense assembly (tiny lattices only)
def dense(apply, n_in: int) -> np.ndarray:
    """Matrix of a linear map by applying it to each unit vector (columns); n_in complex entries."""
    cols = []
    for k in range(n_in):
        e = np.zeros(n_in, dtype=np.complex128)
        e[k] = 1.0
        cols.append(np.asarray(apply(e)).reshape(-1))
    return np.stack(cols, axis=1)
