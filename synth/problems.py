"""Structured-grid FETI test problems (inputs for the oracle and the library).

What is built here is the *problem*, not the method:

* the FEM system K~ u~ = f~ of steady heat conduction or linear elasticity on
  the unit line/square/cube, discretised with linear/bilinear/trilinear
  Lagrange elements on the grid cells, or with linear simplices (triangles,
  tetrahedra: every cell cut into dim! simplices, the paper's element type)
  (paper Sec. II, eq. femsystem);
* its Total-FETI tearing into box subdomains: every subdomain keeps its own
  copy of the interface nodes, gluing between copies and the Dirichlet
  conditions become rows of B with right-hand side c (Sec. II, eqs.
  fetisystemblocked/fetisystem and the Total-FETI remark), so every K_i is
  singular with kernel basis R_i;
* the regularised matrix K_reg,i = K_i + rho * R~_i R~_i^T whose inverse is a
  generalised inverse of K_i (Sec. III: K_i^+ = K_reg,i^{-1}, obtained by
  regularisation); R~_i equals R_i on a few fixing DOFs and is zero elsewhere;
* seeded loads f_i and seeded dual vectors lambda, mu.

Conventions (the paper leaves these open; the readings are fixed here):

* Gluing is non-redundant: a node shared by sorted subdomains s_0<...<s_{k-1}
  gets the chain of rows (s_{t-1}, s_t), t=1..k-1, with +1 on s_{t-1} and -1
  on s_t.  A Dirichlet node gets one row (+1, c=0) on its lowest subdomain.
* Global multiplier order: global nodes ascending (x fastest), per node the
  gluing rows t=1..k-1 then the Dirichlet row, components innermost.  Local
  multipliers of a subdomain are ordered by ascending global index, so the
  dual map D_i is strictly increasing.
* Local DOF order: lexicographic local nodes (x fastest), dof = dpn*node+comp.
* Simplices: the Kuhn subdivision of each cell, one simplex per permutation
  pi of the axes (itertools order) with vertices 0, e_pi0, e_pi0 + e_pi1, ...,
  (1,...,1); neighbouring cells then share their face diagonals.  The dim!
  simplices are images of one another under axis permutations, so with this
  vertex order their heat element matrices coincide.
* rho = max_j (K_i)_jj of the coefficients the problem is generated with; it
  is frozen (a later change of theta keeps rho), so K_reg depends on theta
  only through K_i.
* Heat fixes local node 0; elasticity fixes all components of the corners
  (0,0,0), (w_x,0,0), (0,w_y,0) (2D: (0,0), (w_x,0)).
"""
from __future__ import annotations

import itertools
from dataclasses import dataclass, field

import numpy as np
import scipy.sparse as sp

# --------------------------------------------------------------------------
# reference element matrices (2-point Gauss per axis, exact for these
# multilinear elements on axis-aligned boxes)
# --------------------------------------------------------------------------

_GP = np.array([0.5 - 0.5 / np.sqrt(3.0), 0.5 + 0.5 / np.sqrt(3.0)])
_GW = np.array([0.5, 0.5])


def _corner_offsets(dim):
    """Element corner offsets, lexicographic with x fastest."""
    return np.array([c[::-1] for c in itertools.product((0, 1), repeat=dim)],
                    dtype=np.int64)


def _shape_grads(dim, xi):
    """Gradients of the 2^dim multilinear shape functions on [0,1]^dim at xi.

    Returns an array (2^dim, dim)."""
    corners = _corner_offsets(dim)
    g = np.zeros((len(corners), dim))
    for a, c in enumerate(corners):
        for d in range(dim):
            val = 1.0
            for e in range(dim):
                t = xi[e] if c[e] == 1 else 1.0 - xi[e]
                if e == d:
                    t = 1.0 if c[e] == 1 else -1.0
                val *= t
            g[a, d] = val
    return g


def _elasticity_D(dim, E, nu):
    lam = E * nu / ((1 + nu) * (1 - 2 * nu))
    mu = E / (2 * (1 + nu))
    if dim == 3:
        D = np.zeros((6, 6))
        D[:3, :3] = lam
        D[np.arange(3), np.arange(3)] += 2 * mu
        D[3:, 3:] = np.eye(3) * mu
    elif dim == 2:  # plane strain
        D = np.array([[lam + 2 * mu, lam, 0.0], [lam, lam + 2 * mu, 0.0],
                      [0.0, 0.0, mu]])
    else:
        D = np.array([[E]])
    return D


def _strain_matrix(dim, grads):
    """Voigt strain-displacement matrix for element dofs (dpn*a + comp)."""
    nen = grads.shape[0]
    if dim == 1:
        return grads.T.copy()
    if dim == 2:
        Bm = np.zeros((3, 2 * nen))
        Bm[0, 0::2] = grads[:, 0]
        Bm[1, 1::2] = grads[:, 1]
        Bm[2, 0::2] = grads[:, 1]
        Bm[2, 1::2] = grads[:, 0]
        return Bm
    Bm = np.zeros((6, 3 * nen))
    Bm[0, 0::3] = grads[:, 0]
    Bm[1, 1::3] = grads[:, 1]
    Bm[2, 2::3] = grads[:, 2]
    Bm[3, 0::3] = grads[:, 1]
    Bm[3, 1::3] = grads[:, 0]
    Bm[4, 1::3] = grads[:, 2]
    Bm[4, 2::3] = grads[:, 1]
    Bm[5, 0::3] = grads[:, 2]
    Bm[5, 2::3] = grads[:, 0]
    return Bm


def element_matrix(dim, physics, h=1.0, E=1.0, nu=0.3):
    """Unit-coefficient element stiffness of a box element of edge h.

    heat:        int grad N . grad N^T       (scales as h^(dim-2))
    elasticity:  int B^T D B                  (scales as h^(dim-2))
    """
    nen = 2 ** dim
    dpn = 1 if physics == "heat" else dim
    Ke = np.zeros((nen * dpn, nen * dpn))
    for q in itertools.product(range(2), repeat=dim):
        xi = np.array([_GP[i] for i in q])
        w = np.prod([_GW[i] for i in q])
        g = _shape_grads(dim, xi)
        if physics == "heat":
            Ke += w * g @ g.T
        else:
            Bm = _strain_matrix(dim, g)
            Ke += w * Bm.T @ _elasticity_D(dim, E, nu) @ Bm
    return Ke * h ** (dim - 2)


def kuhn_simplices(dim):
    """Vertex offsets (dim!, dim+1, dim) of the Kuhn simplices of a unit cell."""
    out = []
    for pi in itertools.permutations(range(dim)):
        v = np.zeros(dim, dtype=np.int64)
        verts = [v.copy()]
        for a in pi:
            v[a] += 1
            verts.append(v.copy())
        out.append(np.array(verts))
    return np.array(out)


def simplex_element_matrix(dim, physics, verts, h=1.0, E=1.0, nu=0.3):
    """Unit-coefficient stiffness of the linear simplex with vertex grid
    offsets verts (dim+1, dim) and grid step h: the shape functions are the
    barycentric coordinates, whose gradients are constant."""
    X = np.asarray(verts, dtype=np.float64) * h
    J = (X[1:] - X[0]).T
    Jinv = np.linalg.inv(J)
    g = np.zeros((dim + 1, dim))
    g[1:] = Jinv
    g[0] = -Jinv.sum(axis=0)
    vol = abs(np.linalg.det(J)) / float(np.prod(np.arange(1, dim + 1)))
    if physics == "heat":
        return vol * g @ g.T
    Bm = _strain_matrix(dim, g)
    return vol * Bm.T @ _elasticity_D(dim, E, nu) @ Bm


# --------------------------------------------------------------------------
# data containers
# --------------------------------------------------------------------------


@dataclass
class Subdomain:
    index: int
    dim: int
    dpn: int
    widths: tuple           # elements per axis
    offset: tuple           # global element offset per axis
    coords: np.ndarray      # (nnodes, dim) integer grid coordinates (global)
    gnode: np.ndarray       # (nnodes,) global node id
    elems: np.ndarray       # (ne, 2^dim) local node ids
    gelem: np.ndarray       # (ne,) global element id
    theta: np.ndarray       # (ne,) element coefficients
    Ke_ref: np.ndarray      # unit-coefficient element matrix
    K: sp.csr_matrix        # singular subdomain stiffness
    Kreg: sp.csr_matrix     # regularised stiffness (full symmetric pattern)
    rho: float
    fix_dofs: np.ndarray
    R: np.ndarray           # (n, nk) kernel basis of K
    b_dof: np.ndarray       # (m,) int32 local dof of each local multiplier
    b_sign: np.ndarray      # (m,) int8 +1/-1
    dual_map: np.ndarray    # (m,) int32 global multiplier index, increasing
    f: np.ndarray           # (n,) load
    etype: np.ndarray = None  # (ne,) index into Ke_ref when it stacks several matrices

    @property
    def n(self):
        return self.K.shape[0]

    @property
    def m(self):
        return len(self.b_dof)

    def elem_dofs(self):
        """(ne, nodes per element * dpn) local dofs per element, dof = dpn*node + comp."""
        d = self.dpn
        return (self.elems[:, :, None] * d + np.arange(d)[None, None, :]).reshape(
            self.elems.shape[0], -1)

    @property
    def uniform_elements(self):
        """True when every element has the matrix Ke_ref (nd x nd)."""
        return self.Ke_ref.ndim == 2

    def elem_matrices(self):
        """(ne, nd, nd) unit-coefficient element matrices (a broadcast view
        (1, nd, nd) when they are all equal)."""
        if self.uniform_elements:
            return self.Ke_ref[None, :, :]
        return self.Ke_ref[self.etype]


@dataclass
class Problem:
    name: str
    dim: int
    physics: str
    dpn: int
    h: float
    n_elems: tuple          # global elements per axis
    subs: list
    n_lambda: int
    c: np.ndarray
    lam: np.ndarray
    mu: np.ndarray
    dirichlet_axis: int | None
    meta: dict = field(default_factory=dict)

    @property
    def nsub(self):
        return len(self.subs)


# --------------------------------------------------------------------------
# assembly helpers
# --------------------------------------------------------------------------


def assemble_stiffness(sub: Subdomain, theta=None):
    """K_i = sum_e theta_e * K_e (scattered), as CSR with sorted indices."""
    th = sub.theta if theta is None else np.asarray(theta, dtype=np.float64)
    edofs = sub.elem_dofs()
    ne, nd = edofs.shape
    rows = np.repeat(edofs, nd, axis=1).ravel()
    cols = np.tile(edofs, (1, nd)).ravel()
    vals = (th[:, None, None] * sub.elem_matrices()).ravel()
    n = sub.coords.shape[0] * sub.dpn
    K = sp.coo_matrix((vals, (rows, cols)), shape=(n, n)).tocsr()
    K.sum_duplicates()
    K.sort_indices()
    return K


def regularise(K, R, fix_dofs, rho):
    """K_reg = K + rho * Rt Rt^T with Rt = R restricted to fix_dofs."""
    Rt = R[fix_dofs, :]
    block = rho * (Rt @ Rt.T)
    ii, jj = np.meshgrid(fix_dofs, fix_dofs, indexing="ij")
    n = K.shape[0]
    add = sp.coo_matrix((block.ravel(), (ii.ravel(), jj.ravel())), shape=(n, n))
    Kr = (K + add).tocsr()
    Kr.sum_duplicates()
    Kr.sort_indices()
    return Kr


def _kernel_basis(physics, dim, xyz):
    n = xyz.shape[0]
    if physics == "heat":
        return np.ones((n, 1))
    ctr = xyz.mean(axis=0)
    x = xyz - ctr
    if dim == 1:
        return np.ones((n, 1))
    if dim == 2:
        R = np.zeros((2 * n, 3))
        R[0::2, 0] = 1.0
        R[1::2, 1] = 1.0
        R[0::2, 2] = -x[:, 1]
        R[1::2, 2] = x[:, 0]
        return R
    R = np.zeros((3 * n, 6))
    R[0::3, 0] = 1.0
    R[1::3, 1] = 1.0
    R[2::3, 2] = 1.0
    R[0::3, 3] = -x[:, 1]
    R[1::3, 3] = x[:, 0]
    R[1::3, 4] = -x[:, 2]
    R[2::3, 4] = x[:, 1]
    R[0::3, 5] = x[:, 2]
    R[2::3, 5] = -x[:, 0]
    return R


def _lex_index(c, shape):
    """Lexicographic index, x fastest: c[...,0] + s0*(c[...,1] + s1*c[...,2])."""
    idx = np.zeros(c.shape[:-1], dtype=np.int64)
    for d in reversed(range(len(shape))):
        idx = idx * shape[d] + c[..., d]
    return idx


# --------------------------------------------------------------------------
# the problem builder
# --------------------------------------------------------------------------


def make_problem(dim, physics, widths, theta_sigma=0.0, dirichlet_axis=None,
                 seed=0, E=1.0, nu=0.3, name="custom", elem="box"):
    """Build a torn structured-grid problem.

    widths : list (one per axis) of lists of element counts per subdomain slab.
    theta_sigma : per-element coefficient theta_e = exp(sigma * Z), Z ~ N(0,1)
                  (sigma = 0 gives constant coefficient 1).
    dirichlet_axis : the face {x_axis = 0} carries homogeneous Dirichlet
                  conditions (None: no Dirichlet face).
    seed : int, numpy SeedSequence, or the list of its five spawned
           streams [widths, theta, f, lambda, mu] (the first stream is used by
           config_problem to draw uneven slab widths).
    elem : "box" (multilinear element per grid cell) or "simplex" (dim!
           linear simplices per cell, each with its own coefficient).
    """
    if isinstance(seed, (list, tuple)):
        s_widths, s_theta, s_f, s_lam, s_mu = seed
    else:
        ss = seed if isinstance(seed, np.random.SeedSequence) else np.random.SeedSequence(seed)
        s_widths, s_theta, s_f, s_lam, s_mu = ss.spawn(5)
    assert len(widths) == dim
    widths = [list(map(int, w)) for w in widths]
    dpn = 1 if physics == "heat" else dim
    n_el = tuple(int(sum(w)) for w in widths)
    n_nd = tuple(e + 1 for e in n_el)
    h = 1.0 / max(n_el)
    if elem == "box":
        cell_elems = _corner_offsets(dim)[None]
        Ke_ref = element_matrix(dim, physics, h=h, E=E, nu=nu)
    elif elem == "simplex":
        cell_elems = kuhn_simplices(dim)
        Ke_ref = np.stack([simplex_element_matrix(dim, physics, v, h=h, E=E, nu=nu) for v in cell_elems])
        if np.allclose(Ke_ref, Ke_ref[0], rtol=0.0, atol=1e-14 * np.abs(Ke_ref).max()):
            Ke_ref = Ke_ref[0].copy()
    else:
        raise ValueError(elem)
    per_cell = cell_elems.shape[0]

    # global element coefficients, drawn in global element order so that the
    # field does not depend on the decomposition
    n_gel = int(np.prod(n_el)) * per_cell
    if theta_sigma > 0:
        theta_glob = np.exp(theta_sigma * np.random.default_rng(s_theta).standard_normal(n_gel))
    else:
        theta_glob = np.ones(n_gel)
    rng_f = np.random.default_rng(s_f)

    sub_grid = [len(w) for w in widths]
    offs = [np.concatenate([[0], np.cumsum(w)[:-1]]).astype(int) for w in widths]
    subs = []
    for sidx, sc in enumerate(itertools.product(*[range(s) for s in sub_grid[::-1]])):
        sc = sc[::-1]  # x fastest
        w = tuple(widths[d][sc[d]] for d in range(dim))
        o = tuple(int(offs[d][sc[d]]) for d in range(dim))
        nshape = tuple(x + 1 for x in w)
        lc = np.stack(np.meshgrid(*[np.arange(s) for s in nshape[::-1]], indexing="ij")[::-1],
                      axis=-1).reshape(-1, dim)
        coords = lc + np.array(o)
        gnode = _lex_index(coords, n_nd)
        ec = np.stack(np.meshgrid(*[np.arange(s) for s in w[::-1]], indexing="ij")[::-1],
                      axis=-1).reshape(-1, dim)
        # cell-major, then the cell's elements
        elems = _lex_index(ec[:, None, None, :] + cell_elems[None, :, :, :], nshape).reshape(
            -1, cell_elems.shape[1])
        gelem = (_lex_index(ec + np.array(o), n_el)[:, None] * per_cell
                 + np.arange(per_cell)[None, :]).ravel()
        theta = theta_glob[gelem].copy()
        etype = None if Ke_ref.ndim == 2 else np.tile(np.arange(per_cell), len(ec))
        sub = Subdomain(index=sidx, dim=dim, dpn=dpn, widths=w, offset=o, coords=coords,
                        gnode=gnode, elems=elems, gelem=gelem, theta=theta,
                        Ke_ref=Ke_ref, K=None, Kreg=None, rho=0.0, fix_dofs=None,
                        R=None, b_dof=None, b_sign=None, dual_map=None, f=None, etype=etype)
        sub.K = assemble_stiffness(sub)
        sub.rho = float(sub.K.diagonal().max())
        sub.R = _kernel_basis(physics, dim, coords * h)
        if physics == "heat" or dim == 1:
            fix_nodes = [0]
        else:
            fix_nodes = [0, w[0]] if dim == 2 else [0, w[0], (w[0] + 1) * w[1]]
        sub.fix_dofs = np.array([dpn * a + c for a in fix_nodes for c in range(dpn)],
                                dtype=np.int64)
        sub.Kreg = regularise(sub.K, sub.R, sub.fix_dofs, sub.rho)
        sub.f = rng_f.standard_normal(sub.K.shape[0])
        subs.append(sub)

    # ---- multipliers (gluing chain + Dirichlet rows) ----
    all_g = np.concatenate([s.gnode for s in subs])
    all_s = np.concatenate([np.full(len(s.gnode), s.index) for s in subs])
    all_l = np.concatenate([np.arange(len(s.gnode)) for s in subs])
    order = np.lexsort((all_s, all_g))
    g_s, s_s, l_s = all_g[order], all_s[order], all_l[order]
    uniq, first, cnt = np.unique(g_s, return_index=True, return_counts=True)
    coords_u = np.stack(np.unravel_index(uniq, n_nd[::-1])[::-1], axis=-1)
    if dirichlet_axis is None:
        dflag = np.zeros(len(uniq), dtype=np.int64)
    else:
        dflag = (coords_u[:, dirichlet_axis] == 0).astype(np.int64)
    nrows_node = (cnt - 1) + dflag
    base = np.concatenate([[0], np.cumsum(nrows_node)[:-1]])
    n_noderows = int(nrows_node.sum())
    n_lambda = n_noderows * dpn

    # gluing entries: for positions t>=1 inside each node group
    pos = np.arange(len(g_s)) - np.repeat(first, cnt)
    grp = np.repeat(np.arange(len(uniq)), cnt)
    tmask = pos >= 1
    row_glue = base[grp[tmask]] + pos[tmask] - 1          # node-row index
    idx_t = np.nonzero(tmask)[0]
    ent_sub = np.concatenate([s_s[idx_t - 1], s_s[idx_t]])
    ent_lnode = np.concatenate([l_s[idx_t - 1], l_s[idx_t]])
    ent_row = np.concatenate([row_glue, row_glue])
    ent_sign = np.concatenate([np.ones(len(idx_t)), -np.ones(len(idx_t))])
    # Dirichlet entries: lowest subdomain of the node, row after the gluing rows
    dn = np.nonzero(dflag)[0]
    ent_sub = np.concatenate([ent_sub, s_s[first[dn]]])
    ent_lnode = np.concatenate([ent_lnode, l_s[first[dn]]])
    ent_row = np.concatenate([ent_row, base[dn] + cnt[dn] - 1])
    ent_sign = np.concatenate([ent_sign, np.ones(len(dn))])
    # expand components
    comp = np.arange(dpn)
    e_sub = np.repeat(ent_sub, dpn)
    e_dof = (np.repeat(ent_lnode, dpn) * dpn + np.tile(comp, len(ent_lnode)))
    e_glob = (np.repeat(ent_row, dpn) * dpn + np.tile(comp, len(ent_row)))
    e_sign = np.repeat(ent_sign, dpn)
    o2 = np.lexsort((e_glob, e_sub))
    e_sub, e_dof, e_glob, e_sign = e_sub[o2], e_dof[o2], e_glob[o2], e_sign[o2]
    bounds = np.searchsorted(e_sub, np.arange(len(subs) + 1))
    for s in subs:
        a, b = bounds[s.index], bounds[s.index + 1]
        s.b_dof = e_dof[a:b].astype(np.int32)
        s.b_sign = e_sign[a:b].astype(np.int8)
        s.dual_map = e_glob[a:b].astype(np.int32)
        assert np.all(np.diff(s.dual_map) > 0)

    c = np.zeros(n_lambda)
    lam = np.random.default_rng(s_lam).standard_normal(n_lambda)
    mu = np.random.default_rng(s_mu).standard_normal(n_lambda)
    return Problem(name=name, dim=dim, physics=physics, dpn=dpn, h=h, n_elems=n_el,
                   subs=subs, n_lambda=n_lambda, c=c, lam=lam, mu=mu,
                   dirichlet_axis=dirichlet_axis,
                   meta=dict(theta_sigma=theta_sigma, E=E, nu=nu, elem=elem))


# --------------------------------------------------------------------------
# the five benchmark workloads
# --------------------------------------------------------------------------

CONFIGS = {
    1: "2D heat, unit square, 32x32 bilinear quads in 2x2 subdomains of 16x16, "
       "conductivity 1, Dirichlet x=0",
    2: "3D heat, 96^3 trilinear hexes in 8^3 subdomains of 12^3, "
       "conductivity lognormal(0,0.5), Dirichlet z=0",
    3: "3D elasticity, 9^3 subdomains with seeded slab widths U{6..14}, E=1 nu=0.3, "
       "Dirichlet z=0",
    4: "3D heat, 96^3 hexes in 6^3 subdomains of 16^3, conductivity lognormal(0,1), "
       "Dirichlet z=0",
    5: "3D heat, 40^3 hexes in 4^3 subdomains of 10^3, conductivity exp(N(0,0.3)), "
       "Dirichlet z=0",
}


# the same workloads on linear simplices (every cell cut into dim! simplices)
CONFIGS_SIMPLEX = {
    1: "2D heat, unit square, 32x32 cells x 2 linear triangles in 2x2 subdomains of 16x16 cells, "
       "conductivity 1, Dirichlet x=0",
    2: "3D heat, 96^3 cells x 6 linear tetrahedra in 8^3 subdomains of 12^3 cells, "
       "conductivity lognormal(0,0.5), Dirichlet z=0",
    3: "3D elasticity, linear tetrahedra (6 per cell), 9^3 subdomains with seeded slab widths "
       "U{6..14} cells, E=1 nu=0.3, Dirichlet z=0",
    4: "3D heat, 96^3 cells x 6 linear tetrahedra in 6^3 subdomains of 16^3 cells, "
       "conductivity lognormal(0,1), Dirichlet z=0",
    5: "3D heat, 40^3 cells x 6 linear tetrahedra in 4^3 subdomains of 10^3 cells, "
       "conductivity exp(N(0,0.3)), Dirichlet z=0",
}


def workload_name(k, elem="box"):
    """Description of workload k on box elements or on simplices."""
    return CONFIGS[k] if elem == "box" else CONFIGS_SIMPLEX[k]


def config_problem(k, scale=None, elem="box"):
    """Problem for workload k (1..5), seeded with SeedSequence(1000+k).

    scale : optional (subdomains per axis, elements per subdomain axis) override
            that keeps the workload's physics and coefficient law but shrinks
            the mesh (used for quick tests); None gives the full workload.
    elem :  "box" (the workload's multilinear elements) or "simplex" (the
            same grid cut into linear triangles / tetrahedra).
    """
    ss = list(np.random.SeedSequence(1000 + k).spawn(5))
    kw = dict(elem=elem)
    if k == 1:
        S, W = scale or (2, 16)
        return make_problem(2, "heat", [[W] * S] * 2, 0.0, dirichlet_axis=0, seed=ss,
                            name="C1", **kw)
    if k == 2:
        S, W = scale or (8, 12)
        return make_problem(3, "heat", [[W] * S] * 3, 0.5, dirichlet_axis=2, seed=ss,
                            name="C2", **kw)
    if k == 3:
        S, W = scale or (9, None)
        rng = np.random.default_rng(ss[0])
        if W is None:
            widths = [list(rng.integers(6, 15, size=S)) for _ in range(3)]
        else:
            widths = [[W] * S] * 3
        return make_problem(3, "elasticity", widths, 0.0, dirichlet_axis=2, seed=ss,
                            name="C3", **kw)
    if k == 4:
        S, W = scale or (6, 16)
        return make_problem(3, "heat", [[W] * S] * 3, 1.0, dirichlet_axis=2, seed=ss,
                            name="C4", **kw)
    if k == 5:
        S, W = scale or (4, 10)
        return make_problem(3, "heat", [[W] * S] * 3, 0.3, dirichlet_axis=2, seed=ss,
                            name="C5", **kw)
    raise ValueError(k)
