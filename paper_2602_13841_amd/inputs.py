"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module holds no arithmetic of the method: it only draws random numbers
and lays them out as slab vectors, vertex arrays and smooth random fields.
Both the HIP path and the oracle receive exactly the arrays made here.

Slab vector layout (eq. DefSubvec): U = (V^1..V^{k+1}, P^1..P^{k+1});
V^a = (component 0 nodes, component 1 nodes, ...), nodes of the
((r+1)n+1)^d velocity lattice with x fastest; P^a = (cell 0 modes, cell 1
modes, ...), cells with x fastest.

Recipes (seeded numpy PCG64):
* uniform(-1, 1) vectors for states and directions;
* perturbed meshes: interior vertices of the uniform grid of [0,1]^d moved by
  U(-f h, f h) per coordinate, boundary vertices moved only inside their
  boundary face or edge (corners fixed), so the domain stays [0,1]^d;
* smooth divergence-free random field: v = curl psi (2D: v = (d_y psi,
  -d_x psi)), psi_c(x) = sum_{kappa in {1..m}^d} a_{c,kappa} prod_j
  sin(2 pi kappa_j x_j + phi_{c,j,kappa_j}), a ~ N(0,1)/|kappa|^2, phases
  U(0, 2 pi), scaled to max |v| = 1 over the sample points.  It is sampled
  at the points of the velocity lattice of the unperturbed unit grid (node
  index / (lattice size - 1)): a smooth random state, the same array for
  every consumer.
"""
from __future__ import annotations

from math import comb

import numpy as np


def sizes(dim: int, n, r: int, k: int):
    """(Nv, Np, N) of one slab: velocity and pressure unknowns over all time nodes."""
    n = tuple(int(x) for x in (n if np.ndim(n) else (n,) * dim))[:dim]
    nodes = 1
    cells = 1
    for a in range(dim):
        nodes *= (r + 1) * n[a] + 1
        cells *= n[a]
    nv = dim * nodes
    npr = comb(r + dim, dim) * cells
    return (k + 1) * nv, (k + 1) * npr, (k + 1) * (nv + npr)


def uniform(nvals: int, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    rng = np.random.Generator(np.random.PCG64(seed))
    return rng.uniform(lo, hi, nvals)


def perturbed_vertices(dim: int, n, frac: float, seed: int) -> np.ndarray:
    """Vertices ((n0+1)(n1+1)(n2+1), dim), x fastest, of a randomly perturbed grid."""
    n = tuple(int(x) for x in (n if np.ndim(n) else (n,) * dim))[:dim]
    rng = np.random.Generator(np.random.PCG64(seed))
    axes = [np.arange(n[a] + 1) for a in range(dim)]
    grid = np.meshgrid(*axes, indexing="ij")
    idx = np.stack([g.transpose(tuple(range(dim))[::-1]).ravel() for g in grid], axis=1)
    X = idx / np.array(n, dtype=float)
    h = 1.0 / np.array(n, dtype=float)
    delta = rng.uniform(-frac, frac, X.shape) * h
    onb = (idx == 0) | (idx == np.array(n))
    delta[onb] = 0.0
    return X + delta


def lattice_points(dim: int, n, r: int) -> np.ndarray:
    """Points (Nnodes, dim) of the velocity lattice of the unperturbed unit grid."""
    n = tuple(int(x) for x in (n if np.ndim(n) else (n,) * dim))[:dim]
    N = [(r + 1) * n[a] + 1 for a in range(dim)]
    axes = [np.arange(N[a]) / (N[a] - 1) for a in range(dim)]
    grid = np.meshgrid(*axes, indexing="ij")
    return np.stack([g.transpose(tuple(range(dim))[::-1]).ravel() for g in grid], axis=1)


def fourier_field(points: np.ndarray, seed: int, m: int = 8) -> np.ndarray:
    """Smooth divergence-free random field at `points` (Npts, d) -> (Npts, d)."""
    d = points.shape[1]
    rng = np.random.Generator(np.random.PCG64(seed))
    kap = np.arange(1, m + 1)
    ncomp = 1 if d == 2 else 3
    if d == 2:
        k2 = kap[:, None] ** 2 + kap[None, :] ** 2
    else:
        k2 = kap[:, None, None] ** 2 + kap[None, :, None] ** 2 + kap[None, None, :] ** 2
    amp = rng.standard_normal((ncomp,) + k2.shape) / k2
    phase = rng.uniform(0.0, 2.0 * np.pi, (ncomp, d, m))
    npts = points.shape[0]
    out = np.zeros((npts, d))
    chunk = 1 << 16
    for s0 in range(0, npts, chunk):
        x = points[s0:s0 + chunk]
        # per axis j: f_j[p, kappa] and its derivative
        for c in range(ncomp):
            F = []
            dF = []
            for j in range(d):
                arg = 2.0 * np.pi * x[:, j:j + 1] * kap[None, :] + phase[c, j][None, :]
                F.append(np.sin(arg))
                dF.append(2.0 * np.pi * kap[None, :] * np.cos(arg))
            A = amp[c]
            if d == 2:
                # psi = sum a F0 F1;  v = (d_y psi, -d_x psi)
                dpsi_dx = np.einsum("pi,pj,ij->p", dF[0], F[1], A)
                dpsi_dy = np.einsum("pi,pj,ij->p", F[0], dF[1], A)
                out[s0:s0 + chunk, 0] += dpsi_dy
                out[s0:s0 + chunk, 1] -= dpsi_dx
            else:
                def contract(G0, G1, G2):
                    t = (G0 @ A.reshape(m, m * m)).reshape(-1, m, m)
                    t = np.einsum("pjk,pj->pk", t, G1)
                    return np.einsum("pk,pk->p", t, G2)
                grad = [contract(dF[0], F[1], F[2]), contract(F[0], dF[1], F[2]),
                        contract(F[0], F[1], dF[2])]
                # v = curl psi: v_a += eps_{a b c} d_b psi_c
                if c == 0:
                    out[s0:s0 + chunk, 1] += grad[2]
                    out[s0:s0 + chunk, 2] -= grad[1]
                elif c == 1:
                    out[s0:s0 + chunk, 2] += grad[0]
                    out[s0:s0 + chunk, 0] -= grad[2]
                else:
                    out[s0:s0 + chunk, 0] += grad[1]
                    out[s0:s0 + chunk, 1] -= grad[0]
    return out


def smooth_velocity(dim: int, n, r: int, seed: int, m: int = 8) -> np.ndarray:
    """One time node's velocity vector (component-major) of the smooth field,
    scaled to max |v| = 1."""
    pts = lattice_points(dim, n, r)
    v = fourier_field(pts, seed, m)
    v /= np.max(np.linalg.norm(v, axis=1))
    return np.ascontiguousarray(v.T).ravel()


def slab_state(dim: int, n, r: int, k: int, seed: int, kind: str = "uniform") -> np.ndarray:
    """A full slab vector U used as Newton state.

    kind = "uniform": all entries U(-1,1);
    kind = "smooth": the smooth field at every time node, pressure 0."""
    Nv, Np, N = sizes(dim, n, r, k)
    if kind == "uniform":
        return uniform(N, seed)
    v = smooth_velocity(dim, n, r, seed)
    return np.concatenate([np.tile(v, k + 1), np.zeros(Np)])


def serving_stream(nreq: int, seed: int, dims=(2, 3), ns=(8, 12, 16, 24), rs=(1, 2, 3), ks=(0, 1, 2),
                   res=(1.0, 100.0, 1000.0), tau: float = 1.0 / 64):
    """A mixed stream of slab-solve requests: dimension, cells per axis,
    degrees and Reynolds number drawn uniformly (PCG64, `seed`).  Each request
    is the no-slip problem with zero force whose previous-slab
    velocity is the smooth field (one field per distinct (dim, n, r), seed
    5).  Returns a list of dicts with keys dim, n, r, k, nu, tau, v_prev."""
    rng = np.random.Generator(np.random.PCG64(seed))
    fields = {}
    out = []
    for _ in range(nreq):
        d = int(rng.choice(dims))
        n = int(rng.choice(ns))
        r = int(rng.choice(rs))
        k = int(rng.choice(ks))
        re = float(rng.choice(res))
        key = (d, n, r)
        if key not in fields:
            fields[key] = smooth_velocity(d, (n,) * d, r, 5)
        out.append(dict(dim=d, n=(n,) * d, r=r, k=k, nu=1.0 / re, tau=tau, v_prev=fields[key]))
    return out


def poisson_arrivals(nreq: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (s) of a Poisson process of the given rate."""
    rng = np.random.Generator(np.random.PCG64(seed))
    return np.cumsum(rng.exponential(1.0 / rate, nreq))
