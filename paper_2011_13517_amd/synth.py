"""Seeded synthetic inputs for the spectral-quadrature density path.

This module only *builds inputs*: a finite-difference grid, a local potential
sampled on it, nonlocal projector tables, node lists and truncation widths.
It holds none of the method's arithmetic (no Hamiltonian, no recurrence, no
coefficients), so both the CPU oracle and the HIP library may consume what it
produces.

The workloads stand in for the paper's magnesium / magnesium-aluminium cells
(Section 4 and Section 5; hcp Mg lattice a = 6.043, c = 9.848 bohr), which need
Troullier-Martins pseudopotential data that is not available.  Instead:

* the local potential is a sum of negative Gaussians, one per atom
  (depth D ~ U(0.5, 1.5) Ha, Al solutes D ~ U(1.5, 2.5) Ha, width sigma = 1 bohr);
* each atom carries four Kleinman-Bylander style projectors (s, px, py, pz)
  with a Gaussian radial part and a C1 taper that vanishes at r_c = 2.5 bohr:
  chi_s = N_0 f(r), chi_pa = N_1 d_a f(r),
  f(r) = exp(-r^2 / (2 sigma_p^2)) (1 - (r/r_c)^2)^2,  sigma_p = r_c / 3,
  with N_l the continuum normalisation (integral of chi^2 over space is 1);
* projector energies c_Jl = +-U(0.1, 1) Ha, sign drawn per (atom, l).

Grid conventions (shared by every consumer): node (i, j, k) sits at
x = (i*h0, j*h1, k*h2) bohr; arrays are flattened with i fastest,
idx = i + n0*(j + n1*k).  For the embedded boundary mode the potential and the
projector supports live on the padded grid Omega' whose node i' sits at
x = (i' - pad) * h.

Boundary modes: 0 = periodic, 1 = Dirichlet (regions clipped at the domain
boundary, zero outside), 2 = embedded (potential given on Omega').
"""
from __future__ import annotations

import dataclasses
from typing import Optional

import numpy as np

BC_PERIODIC, BC_DIRICHLET, BC_EMBEDDED = 0, 1, 2

# orthorhombic 4-site hcp-like basis, fractional coordinates of the cell
HCP_BASIS = np.array([[0.0, 0.0, 0.0],
                      [0.5, 0.5, 0.0],
                      [0.5, 1.0 / 6.0, 0.5],
                      [0.0, 2.0 / 3.0, 0.5]])


@dataclasses.dataclass
class Problem:
    """Everything a density evaluation needs, as plain numpy arrays."""
    name: str
    n: tuple            # Omega grid (n0, n1, n2)
    h: tuple            # spacing (bohr)
    fd_order: int       # even; FD radius r = fd_order // 2
    bc: int             # BC_* mode
    rcut: tuple         # default half-width of a node region, in nodes per axis
    order: int          # Chebyshev degree K
    kT: float           # smearing (Ha)
    V: np.ndarray       # local potential, float64, flattened over Omega or Omega'
    Ne: Optional[float] = None        # electron count (None: lambda_f is fixed)
    lambda_f: Optional[float] = None  # fixed Fermi level when Ne is None
    # projector tables (CSR over atoms); n_atoms == 0 means no nonlocal term
    n_atoms: int = 0
    n_proj: int = 4
    sup_off: Optional[np.ndarray] = None   # int64 [n_atoms+1]
    sup_idx: Optional[np.ndarray] = None   # int64 [nnz], linear index in V's grid
    chi: Optional[np.ndarray] = None       # float64 [nnz, n_proj]
    dchi: Optional[np.ndarray] = None      # float64 [nnz, n_proj, 3] = d chi / d R_J
    c: Optional[np.ndarray] = None         # float64 [n_atoms, n_proj]
    atom_pos: Optional[np.ndarray] = None  # float64 [n_atoms, 3] (bohr, Omega frame)
    # node set: None means every node of Omega, in linear order
    nodes: Optional[np.ndarray] = None     # int64 [n_nodes]
    node_rcut: Optional[np.ndarray] = None  # int32 [n_nodes, 3]
    precision: int = 0  # 0 = FP64, 1 = FP32 recurrence with FP64 moments

    @property
    def r(self) -> int:
        return self.fd_order // 2

    @property
    def pad(self) -> tuple:
        return tuple(self.rcut) if self.bc == BC_EMBEDDED else (0, 0, 0)

    @property
    def vshape(self) -> tuple:
        p = self.pad
        return tuple(int(self.n[a] + 2 * p[a]) for a in range(3))

    @property
    def n_nodes(self) -> int:
        if self.nodes is None:
            return int(np.prod(self.n))
        return int(self.nodes.shape[0])

    def node_list(self) -> np.ndarray:
        if self.nodes is None:
            return np.arange(int(np.prod(self.n)), dtype=np.int64)
        return self.nodes

    def node_widths(self) -> np.ndarray:
        if self.node_rcut is None:
            return np.tile(np.asarray(self.rcut, dtype=np.int32), (self.n_nodes, 1))
        return self.node_rcut

    def with_nodes(self, nodes, node_rcut=None) -> "Problem":
        return dataclasses.replace(self, nodes=np.asarray(nodes, dtype=np.int64),
                                   node_rcut=None if node_rcut is None
                                   else np.asarray(node_rcut, dtype=np.int32))


# --------------------------------------------------------------------------- #
# lattices
# --------------------------------------------------------------------------- #
def hcp_sites(cells, edges, jitter, rng):
    """Sites of cells[0] x cells[1] x cells[2] orthorhombic 4-site cells."""
    ijk = np.stack(np.meshgrid(*[np.arange(c) for c in cells], indexing="ij"), -1).reshape(-1, 3)
    frac = (ijk[:, None, :] + HCP_BASIS[None, :, :]).reshape(-1, 3)
    pos = frac * np.asarray(edges)[None, :]
    if jitter > 0:
        pos = pos + rng.normal(0.0, jitter, size=pos.shape)
    return pos


# --------------------------------------------------------------------------- #
# fields on the grid
# --------------------------------------------------------------------------- #
def _axis_coords(n, h, pad):
    return [(np.arange(n[a] + 2 * pad[a]) - pad[a]) * h[a] for a in range(3)]


def gaussian_potential(n, h, pad, centers, depths, sigma, periodic_len=None, cutoff=9.0):
    """V(x) = -sum_J D_J exp(-|x - R_J|^2 / (2 sigma^2)) on the (padded) grid.

    periodic_len: box lengths; when given, every periodic image whose Gaussian
    reaches the grid (within `cutoff` sigmas) is added."""
    shape = tuple(n[a] + 2 * pad[a] for a in range(3))
    V = np.zeros(shape[::-1], dtype=np.float64)   # [k][j][i]
    ax = _axis_coords(n, h, pad)
    rmax = cutoff * sigma
    lo = [ax[a][0] for a in range(3)]
    hi = [ax[a][-1] for a in range(3)]
    for R, D in zip(centers, depths):
        shifts = [[0.0] for _ in range(3)]
        if periodic_len is not None:
            for a in range(3):
                L = periodic_len[a]
                kmin = int(np.floor((lo[a] - rmax - R[a]) / L))
                kmax = int(np.ceil((hi[a] + rmax - R[a]) / L))
                shifts[a] = [k * L for k in range(kmin, kmax + 1)]
        for sx in shifts[0]:
            for sy in shifts[1]:
                for sz in shifts[2]:
                    c = (R[0] + sx, R[1] + sy, R[2] + sz)
                    sl = []
                    ok = True
                    for a in range(3):
                        i0 = int(np.ceil((c[a] - rmax) / h[a])) + pad[a]
                        i1 = int(np.floor((c[a] + rmax) / h[a])) + pad[a]
                        i0 = max(i0, 0)
                        i1 = min(i1, shape[a] - 1)
                        if i0 > i1:
                            ok = False
                            break
                        sl.append((i0, i1))
                    if not ok:
                        continue
                    gx = ax[0][sl[0][0]:sl[0][1] + 1] - c[0]
                    gy = ax[1][sl[1][0]:sl[1][1] + 1] - c[1]
                    gz = ax[2][sl[2][0]:sl[2][1] + 1] - c[2]
                    r2 = gz[:, None, None] ** 2 + gy[None, :, None] ** 2 + gx[None, None, :] ** 2
                    V[sl[2][0]:sl[2][1] + 1, sl[1][0]:sl[1][1] + 1, sl[0][0]:sl[0][1] + 1] -= \
                        D * np.exp(-r2 / (2.0 * sigma * sigma))
    return V.reshape(-1)


def _radial_norms(rc, sigma_p):
    """Continuum normalisation constants N_0, N_1 of the tapered Gaussian projectors."""
    r = np.linspace(0.0, rc, 200001)
    f = np.exp(-r * r / (2 * sigma_p * sigma_p)) * (1 - (r / rc) ** 2) ** 2
    i0 = 4 * np.pi * np.trapezoid(f * f * r * r, r)
    i1 = 4 * np.pi / 3 * np.trapezoid(f * f * r ** 4, r)
    return 1.0 / np.sqrt(i0), 1.0 / np.sqrt(i1)


def projector_tables(n, h, pad, centers, mode, rc=2.5, periodic_len=None):
    """CSR projector tables (s, px, py, pz) for atoms at `centers`.

    mode: BC_* of the grid; periodic grids wrap the support, the other modes
    keep only support points on the (padded) grid.  Returns
    (sup_off, sup_idx, chi, dchi) with dchi = d chi / d R_J = -grad_x chi."""
    sigma_p = rc / 3.0
    N0, N1 = _radial_norms(rc, sigma_p)
    shape = tuple(n[a] + 2 * pad[a] for a in range(3))
    offs = [0]
    idx_l, chi_l, dchi_l = [], [], []
    for R in centers:
        rng_ax = []
        for a in range(3):
            i0 = int(np.floor((R[a] - rc) / h[a])) - 1
            i1 = int(np.ceil((R[a] + rc) / h[a])) + 1
            rng_ax.append(np.arange(i0, i1 + 1))
        I, J, K = np.meshgrid(*rng_ax, indexing="ij")
        I, J, K = I.ravel(order="F"), J.ravel(order="F"), K.ravel(order="F")
        d = np.stack([I * h[0] - R[0], J * h[1] - R[1], K * h[2] - R[2]], -1)
        r2 = (d * d).sum(-1)
        keep = r2 < rc * rc
        I, J, K, d, r2 = I[keep], J[keep], K[keep], d[keep], r2[keep]
        gi = np.stack([I + pad[0], J + pad[1], K + pad[2]], -1)
        if mode == BC_PERIODIC:
            gi = gi % np.asarray(shape)[None, :]
        else:
            inside = np.all((gi >= 0) & (gi < np.asarray(shape)[None, :]), axis=1)
            gi, d, r2 = gi[inside], d[inside], r2[inside]
        lin = gi[:, 0] + shape[0] * (gi[:, 1] + shape[1] * gi[:, 2])
        order = np.argsort(lin, kind="stable")
        lin, d, r2 = lin[order], d[order], r2[order]
        t2 = r2 / (rc * rc)
        e = np.exp(-r2 / (2 * sigma_p * sigma_p))
        f = e * (1 - t2) ** 2
        g = e * (1 - t2) * (-(1 - t2) / (sigma_p * sigma_p) - 4.0 / (rc * rc))  # f'(r)/r
        chi = np.empty((lin.size, 4))
        chi[:, 0] = N0 * f
        chi[:, 1:] = N1 * d * f[:, None]
        grad = np.empty((lin.size, 4, 3))
        grad[:, 0, :] = N0 * d * g[:, None]
        for a in range(3):
            grad[:, 1 + a, :] = N1 * d[:, a:a + 1] * d * g[:, None]
            grad[:, 1 + a, a] += N1 * f
        idx_l.append(lin.astype(np.int64))
        chi_l.append(chi)
        dchi_l.append(-grad)
        offs.append(offs[-1] + lin.size)
    if not centers.shape[0]:
        return (np.zeros(1, np.int64), np.zeros(0, np.int64), np.zeros((0, 4)), np.zeros((0, 4, 3)))
    return (np.asarray(offs, np.int64), np.concatenate(idx_l), np.concatenate(chi_l),
            np.concatenate(dchi_l))


def projector_energies(n_atoms, rng):
    mag = rng.uniform(0.1, 1.0, size=(n_atoms, 2))
    sgn = np.where(rng.uniform(size=(n_atoms, 2)) < 0.5, -1.0, 1.0)
    cl = mag * sgn
    return np.stack([cl[:, 0], cl[:, 1], cl[:, 1], cl[:, 1]], -1)


# --------------------------------------------------------------------------- #
# generic builder
# --------------------------------------------------------------------------- #
def build_problem(name, n, h, fd_order, bc, rcut, order, kT, centers, depths, *,
                  sigma=1.0, proj_centers=None, rng=None, with_projectors=True,
                  rc=2.5, Ne=None, lambda_f=None, periodic_images=True):
    """Assemble a Problem from atom centres (bohr) and Gaussian depths (Ha)."""
    rng = rng if rng is not None else np.random.default_rng(0)
    n = tuple(int(x) for x in n)
    h = tuple(float(x) for x in h)
    rcut = tuple(int(x) for x in rcut)
    pad = rcut if bc == BC_EMBEDDED else (0, 0, 0)
    L = tuple(n[a] * h[a] for a in range(3))
    V = gaussian_potential(n, h, pad, centers, depths, sigma,
                           periodic_len=L if (bc == BC_PERIODIC and periodic_images) else None)
    prob = Problem(name=name, n=n, h=h, fd_order=fd_order, bc=bc, rcut=rcut, order=order,
                   kT=kT, V=V, Ne=Ne, lambda_f=lambda_f)
    if with_projectors:
        pc = centers if proj_centers is None else proj_centers
        off, idx, chi, dchi = projector_tables(n, h, pad, pc, bc, rc=rc)
        prob.n_atoms = int(pc.shape[0])
        prob.sup_off, prob.sup_idx, prob.chi, prob.dchi = off, idx, chi, dchi
        prob.c = projector_energies(prob.n_atoms, rng)
        prob.atom_pos = np.asarray(pc, dtype=np.float64)
    return prob


# --------------------------------------------------------------------------- #
# the five workloads
# --------------------------------------------------------------------------- #
def config(c: int) -> Problem:
    """Workload c (1..5); seeds are numpy default_rng(1000 + c)."""
    rng = np.random.default_rng(1000 + c)
    if c == 1:
        # 12^3 periodic, h = 0.5, 4th-order FD, 8 Gaussians, 9^3 regions, K = 40, local only
        n, h = (12, 12, 12), (0.5, 0.5, 0.5)
        depths = rng.uniform(0.5, 1.5, size=8)
        centers = rng.uniform(0.0, 6.0, size=(8, 3))
        return build_problem("c1_periodic12_r2_K40", n, h, 4, BC_PERIODIC, (4, 4, 4), 40, 0.005,
                             centers, depths, rng=rng, with_projectors=False, Ne=16.0)
    if c in (2, 3):
        rng2 = np.random.default_rng(1002)
        n, h = (64, 64, 64), (0.45, 0.45, 0.45)
        centers = hcp_sites((4, 3, 2), (7.2, 9.6, 14.4), 0.05, rng2) % 28.8
        depths = rng2.uniform(0.5, 1.5, size=centers.shape[0])
        if c == 2:
            return build_problem("c2_periodic64_r6_K100_nl", n, h, 12, BC_PERIODIC, (13, 13, 13),
                                 100, 0.001, centers, depths, rng=rng2, Ne=192.0)
        # config 3: same potential, non-periodic domain, 4096 uneven clipped regions
        prob = build_problem("c3_dirichlet64_uneven_K100", n, h, 12, BC_DIRICHLET, (13, 13, 13),
                             100, 0.001, centers, depths, rng=rng2, lambda_f=FIXED_LAMBDA_F_C3)
        # the potential itself is config 2's periodic sum
        prob.V = gaussian_potential(n, h, (0, 0, 0), centers, depths, 1.0,
                                    periodic_len=(28.8, 28.8, 28.8))
        nodes = rng.choice(int(np.prod(n)), size=4096, replace=False).astype(np.int64)
        m = rng.integers(5, 14, size=4096).astype(np.int32)
        return prob.with_nodes(nodes, np.repeat(m[:, None], 3, axis=1))
    if c == 4:
        n, h = (48, 48, 48), (0.45, 0.45, 0.45)
        L = 21.6
        sites = hcp_sites((4, 2, 2), (5.4, 10.8, 10.8), 0.05, rng) % L
        vac = int(rng.integers(0, sites.shape[0]))
        centers = np.delete(sites, vac, axis=0)
        depths = rng.uniform(0.5, 1.5, size=centers.shape[0])
        return build_problem("c4_periodic48_r6_K80_vacancy", n, h, 12, BC_PERIODIC, (10, 10, 10),
                             80, 0.002, centers, depths, rng=rng, Ne=126.0)
    if c == 5:
        return _config5(rng)
    raise ValueError(f"unknown config {c}")


def without_projectors(prob: Problem) -> Problem:
    """The same grid, potential, nodes and regions with no nonlocal term: the
    local part of the Hamiltonian alone (used to time the stencil and diagonal
    apart from the projector block)."""
    return dataclasses.replace(prob, name=prob.name + "_local", n_atoms=0, sup_off=None,
                               sup_idx=None, chi=None, dchi=None, c=None, atom_pos=None)


# lambda_f used by the uneven-region workload, which has no electron count of its
# own: the FP64 Fermi level of the 64^3 workload (config 2), computed by the oracle
# alone over all of its nodes (tests/golden/make_c2_lambda_f.py -> c2_lambda_f.txt)
FIXED_LAMBDA_F_C3 = 0.09726053266210105


def _config5(rng):
    """128^3 embedded domain, 2x2x2 replica of the 96-site cell, 2 Al + divacancy."""
    n, h = (128, 128, 128), (0.45, 0.45, 0.45)
    m = 13
    Lc = 28.8
    rng2 = np.random.default_rng(1002)
    base = hcp_sites((4, 3, 2), (7.2, 9.6, 14.4), 0.05, rng2) % Lc
    base_depth = rng2.uniform(0.5, 1.5, size=base.shape[0])
    L = 2 * Lc
    shifts = np.array([[i, j, k] for i in range(2) for j in range(2) for k in range(2)], float) * Lc
    sites = (base[None, :, :] + shifts[:, None, :]).reshape(-1, 3)
    depth = np.tile(base_depth, 8)
    z = np.full(sites.shape[0], 2.0)
    center = np.array([L / 2] * 3)
    d0 = np.linalg.norm(sites - center, axis=1)
    al1 = int(np.argmin(d0))
    dd = np.linalg.norm(sites - sites[al1], axis=1)
    dd[al1] = np.inf
    al2 = int(np.argmin(dd))
    nn = dd[al2]
    depth[[al1, al2]] = rng.uniform(1.5, 2.5, size=2)
    z[[al1, al2]] = 3.0
    # divacancy: a first-neighbour pair at least three neighbour distances from both solutes
    far = (np.linalg.norm(sites - sites[al1], axis=1) >= 3 * nn) & \
          (np.linalg.norm(sites - sites[al2], axis=1) >= 3 * nn)
    cand = np.flatnonzero(far)
    rng.shuffle(cand)
    pair = None
    for a in cand:
        dist = np.linalg.norm(sites - sites[a], axis=1)
        dist[a] = np.inf
        b = int(np.argmin(dist))
        if far[b] and dist[b] < 1.05 * nn:
            pair = (int(a), b)
            break
    keep = np.ones(sites.shape[0], bool)
    keep[list(pair)] = False
    in_sites, in_depth, in_z = sites[keep], depth[keep], z[keep]
    # perfect-crystal continuation outside Omega (periodic images of the defect-free lattice)
    pad_b = m * h[0] + 9.0
    img = []
    img_depth = []
    for sx in (-1, 0, 1):
        for sy in (-1, 0, 1):
            for sz in (-1, 0, 1):
                if sx == sy == sz == 0:
                    continue
                p = sites + np.array([sx, sy, sz]) * L
                ok = np.all((p > -pad_b) & (p < L + pad_b), axis=1)
                img.append(p[ok])
                img_depth.append(np.tile(base_depth, 8)[ok])
    out_sites = np.concatenate(img)
    out_depth = np.concatenate(img_depth)
    all_sites = np.concatenate([in_sites, out_sites])
    all_depth = np.concatenate([in_depth, out_depth])
    # projectors only for atoms whose support reaches Omega'
    rc = 2.5
    lo, hi = -m * h[0] - rc, L + (m - 1) * h[0] + rc
    touch = np.all((all_sites > lo) & (all_sites < hi), axis=1)
    prob = build_problem("c5_embedded128_r6_K120_defects", n, h, 12, BC_EMBEDDED, (m, m, m), 120,
                         0.001, all_sites, all_depth, proj_centers=all_sites[touch], rng=rng,
                         Ne=float(in_z.sum()), periodic_images=False)
    return prob


def pseudocharge(prob: Problem, Z=None, sigma=1.0) -> np.ndarray:
    """Seeded stand-in for the nuclei's pseudocharge density b(x): a normalised
    Gaussian of charge -Z_J per atom.  Periodic grids sum the periodic images and
    rescale so that sum_x b(x) h1 h2 h3 = -sum_J Z_J exactly (the cell is neutral
    once the electrons are added); embedded grids give b on Omega' (no images,
    no rescaling).  Z defaults to 2 per atom."""
    assert prob.bc in (BC_PERIODIC, BC_EMBEDDED) and prob.atom_pos is not None
    Z = np.full(prob.n_atoms, 2.0) if Z is None else np.asarray(Z, dtype=np.float64)
    norm = (2.0 * np.pi * sigma * sigma) ** -1.5
    if prob.bc == BC_EMBEDDED:
        return gaussian_potential(prob.n, prob.h, prob.pad, prob.atom_pos, Z * norm, sigma)
    L = [prob.n[a] * prob.h[a] for a in range(3)]
    b = gaussian_potential(prob.n, prob.h, (0, 0, 0), prob.atom_pos, Z * norm, sigma,
                           periodic_len=L)
    h3 = float(np.prod(prob.h))
    return b * (Z.sum() / (-b.sum() * h3))


def small_problem(seed, n=(8, 8, 8), h=(0.6, 0.6, 0.6), fd_order=4, bc=BC_PERIODIC,
                  rcut=(2, 2, 2), order=12, kT=0.1, n_atoms=3, with_projectors=True, rc=1.3,
                  Ne=None):
    """Tiny randomized problem for oracle pins and parity on several tiles."""
    rng = np.random.default_rng(seed)
    L = np.array([n[a] * h[a] for a in range(3)])
    centers = rng.uniform(0.0, 1.0, size=(n_atoms, 3)) * L
    depths = rng.uniform(0.5, 1.5, size=n_atoms)
    prob = build_problem(f"small{seed}", n, h, fd_order, bc, rcut, order, kT, centers, depths,
                         rng=rng, with_projectors=with_projectors, rc=rc, Ne=Ne,
                         sigma=1.0)
    return prob
