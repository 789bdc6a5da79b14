"""Seeded synthetic patch batches for the FV patch-update workloads.

This module only draws input states; it contains none of the update's
arithmetic, and both the GPU path and the CPU oracle consume what it returns.

Layout of a batch (the layout the library's C ABI takes): one flat float64
array; patch t starts at ``offsets[t]`` (in doubles) and holds its
(p_t + 2)^d volumes in x-fastest order, each volume its N unknowns
contiguously (array of structures), halo volumes at index 0 and p_t + 1 of
every axis.

State recipe (the paper fixes no initial data; these draws stand in for the
patches an ExaHyPE traversal would hand the kernel):
  * primitives drawn i.i.d. per volume (interior and halo alike):
    rho ~ U[0.5, 1.5], u, v, w ~ U[-0.5, 0.5], p ~ U[0.5, 1.5];
  * optionally a smooth Gaussian density pulse per patch,
    rho += 0.1 exp(-|x - x_c|^2 / (2 sigma^2)), x_c the patch centre,
    sigma = p h / 4, added before the conversion to conserved variables;
  * conserved variables: (rho, rho u, rho v[, rho w], E) with
    E = p / (gamma - 1) + rho |u|^2 / 2 (w is stored when N = 5, also in 2D).
Draw order with ``numpy.random.Generator(PCG64(seed))``: the patch sizes
(mixed batches only), then rho, u, v, w, p over all volumes of all patches in
patch order.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np

GAMMA = 1.4
H_DEFAULT = 1.0 / 48.0
CFL = 0.4


@dataclass
class Batch:
    """A flat batch of halo-padded patches."""

    data: np.ndarray      # float64 [total doubles]
    sizes: np.ndarray     # int32 [T], interior volumes per axis
    offsets: np.ndarray   # int64 [T], start of each patch in doubles
    dim: int
    nq: int

    @property
    def num_patches(self) -> int:
        return int(self.sizes.shape[0])

    @property
    def uniform(self) -> bool:
        return bool(self.num_patches == 0 or np.all(self.sizes == self.sizes[0]))

    def patch_volumes(self) -> np.ndarray:
        return (self.sizes.astype(np.int64) + 2) ** self.dim

    def interior_volumes(self) -> int:
        return int(np.sum(self.sizes.astype(np.int64) ** self.dim))

    def patch(self, t: int) -> np.ndarray:
        """View of patch t as an array [(p+2)]*dim reversed (k, j, i) x nq."""
        p = int(self.sizes[t])
        n = (p + 2) ** self.dim * self.nq
        shape = (p + 2,) * self.dim + (self.nq,)
        return self.data[self.offsets[t]:self.offsets[t] + n].reshape(shape)


def contiguous_offsets(sizes: np.ndarray, dim: int, nq: int) -> np.ndarray:
    vols = (np.asarray(sizes, dtype=np.int64) + 2) ** dim * nq
    off = np.zeros(len(vols), dtype=np.int64)
    if len(vols) > 1:
        off[1:] = np.cumsum(vols)[:-1]
    return off


def _draw_primitives(rng: np.random.Generator, nvol: int):
    rho = rng.uniform(0.5, 1.5, nvol)
    u = rng.uniform(-0.5, 0.5, nvol)
    v = rng.uniform(-0.5, 0.5, nvol)
    w = rng.uniform(-0.5, 0.5, nvol)
    p = rng.uniform(0.5, 1.5, nvol)
    return rho, u, v, w, p


def _pulse(sizes: np.ndarray, dim: int, h: float) -> np.ndarray:
    """Gaussian density pulse, one per patch, centred on the patch centre."""
    parts = []
    for p in np.unique(sizes):
        p = int(p)
        idx = (np.arange(p + 2) - (p + 1) / 2.0) * h
        grids = np.meshgrid(*([idx] * dim), indexing="ij")
        r2 = sum(g * g for g in grids)
        sigma = p * h / 4.0
        parts.append((p, (0.1 * np.exp(-r2 / (2.0 * sigma * sigma))).reshape(-1)))
    table = dict(parts)
    return np.concatenate([table[int(p)] for p in sizes]) if len(sizes) else np.zeros(0)


def conserved(rho, u, v, w, p, nq: int, gamma: float = GAMMA) -> np.ndarray:
    """Stack primitive draws into conserved AoS volumes [nvol, nq]."""
    ke = 0.5 * rho * (u * u + v * v + (w * w if nq == 5 else 0.0))
    E = p / (gamma - 1.0) + ke
    cols = [rho, rho * u, rho * v] + ([rho * w] if nq == 5 else []) + [E]
    return np.stack(cols, axis=1)


def make_batch(sizes, dim: int = 2, nq: int = 5, seed: int = 0, pulse: bool = False,
               h: float = H_DEFAULT, gamma: float = GAMMA, rng: np.random.Generator | None = None) -> Batch:
    """Contiguous batch of patches with the given interior sizes."""
    sizes = np.asarray(sizes, dtype=np.int32)
    rng = rng if rng is not None else np.random.Generator(np.random.PCG64(seed))
    nvol = int(np.sum((sizes.astype(np.int64) + 2) ** dim))
    rho, u, v, w, p = _draw_primitives(rng, nvol)
    if pulse:
        rho = rho + _pulse(sizes, dim, h)
    data = conserved(rho, u, v, w, p, nq, gamma).reshape(-1).copy()
    return Batch(data=data, sizes=sizes, offsets=contiguous_offsets(sizes, dim, nq), dim=dim, nq=nq)


def make_uniform(num_patches: int, p: int, dim: int = 2, nq: int = 5, seed: int = 0, pulse: bool = False,
                 h: float = H_DEFAULT, gamma: float = GAMMA) -> Batch:
    return make_batch(np.full(num_patches, p, dtype=np.int32), dim, nq, seed, pulse, h, gamma)


def make_mixed(num_patches: int, choices=(3, 5, 9, 17), dim: int = 2, nq: int = 5, seed: int = 0,
               pulse: bool = False, h: float = H_DEFAULT, gamma: float = GAMMA) -> Batch:
    """Patch sizes drawn uniformly from ``choices`` (drawn first), then the state."""
    rng = np.random.Generator(np.random.PCG64(seed))
    sizes = rng.choice(np.asarray(choices, dtype=np.int32), size=num_patches)
    return make_batch(sizes, dim, nq, seed, pulse, h, gamma, rng=rng)


# Named workloads.  Each entry: (builder kwargs, steps, periodic halo write).
# ---------------------------------------------------------------- patch meshes
# A conforming Cartesian mesh of n^d patches of one size covering the unit
# square / cube, stored in the order of a space-filling curve over the patch
# grid (Peano for n = 3^k in 2D, Morton for n = 2^k, row-major otherwise).
# Only topology: which patch sits where and which patch touches which face.


def _peano2d(n: int):
    """Cells (x, y) of an n x n grid, n = 3^k, in Peano-curve order: columns of
    3 x 3 blocks traversed bottom-up, top-down, bottom-up, each block
    reflected so that consecutive cells share a face."""
    if n == 1:
        return [(0, 0)]
    m = n // 3
    sub = _peano2d(m)
    out = []
    for bi in range(3):
        rows = range(3) if bi % 2 == 0 else range(2, -1, -1)
        for vis, bj in enumerate(rows):
            flip_x = vis % 2 == 1
            flip_y = bi % 2 == 1
            for (x, y) in sub:
                xx = m - 1 - x if flip_x else x
                yy = m - 1 - y if flip_y else y
                out.append((bi * m + xx, bj * m + yy))
    return out


def _morton(n: int, dim: int):
    cells = []
    bits = n.bit_length() - 1
    for code in range(n ** dim):
        c = [0] * dim
        for b in range(bits):
            for a in range(dim):
                c[a] |= ((code >> (b * dim + a)) & 1) << b
        cells.append(tuple(c))
    return cells


def mesh_order(n: int, dim: int):
    """Patch grid coordinates in storage order."""
    if dim == 2 and n >= 3 and 3 ** round(np.log(n) / np.log(3)) == n:
        return _peano2d(n)
    if n >= 2 and n & (n - 1) == 0:
        return _morton(n, dim)
    if dim == 2:
        return [(x, y) for y in range(n) for x in range(n)]
    return [(x, y, z) for z in range(n) for y in range(n) for x in range(n)]


@dataclass
class Mesh:
    batch: Batch
    n: int                 # patches per axis
    coords: np.ndarray     # int32 [T, dim]: grid position of patch t
    neighbors: np.ndarray  # int32 [T, 2 dim]: patch across face (axis a, side s) at 2 a + s, or -1
    periodic: bool

    @property
    def h(self) -> float:
        """Volume width of the unit domain."""
        return 1.0 / (self.n * int(self.batch.sizes[0]))


def make_mesh(n: int, p: int, dim: int = 2, nq: int = 5, seed: int = 0, periodic: bool = True,
              pulse: bool = False) -> Mesh:
    """n^d patches of p^d volumes in space-filling-curve order with their
    face-neighbour table (wrapping around when periodic, -1 at the boundary
    otherwise); states drawn as in make_uniform."""
    cells = mesh_order(n, dim)
    T = len(cells)
    index = {c: t for t, c in enumerate(cells)}
    nb = np.full((T, 2 * dim), -1, np.int32)
    for t, c in enumerate(cells):
        for a in range(dim):
            for s, step in ((0, -1), (1, 1)):
                q = list(c)
                q[a] += step
                if not 0 <= q[a] < n:
                    if not periodic:
                        continue
                    q[a] %= n
                nb[t, 2 * a + s] = index[tuple(q)]
    batch = make_uniform(T, p, dim=dim, nq=nq, seed=seed, pulse=pulse)
    return Mesh(batch=batch, n=n, coords=np.asarray(cells, np.int32), neighbors=nb, periodic=periodic)


WORKLOADS = {
    "c1_2d_p3_T16": dict(kind="uniform", num_patches=16, p=3, dim=2, steps=1, periodic=False, pulse=False),
    "c2_2d_p16_T65536": dict(kind="uniform", num_patches=65536, p=16, dim=2, steps=10, periodic=True, pulse=True),
    "c3_2d_mixed_T200000": dict(kind="mixed", num_patches=200000, choices=(3, 5, 9, 17), dim=2, steps=10,
                                periodic=False, pulse=False),
    "c4_3d_p8_T32768": dict(kind="uniform", num_patches=32768, p=8, dim=3, steps=10, periodic=False, pulse=False),
}


def build_workload(name: str, seed: int = 0, num_patches: int | None = None, nq: int = 5) -> tuple[Batch, dict]:
    """Build a named workload (optionally with fewer patches for parity runs)."""
    spec = dict(WORKLOADS[name])
    T = num_patches if num_patches is not None else spec["num_patches"]
    if spec["kind"] == "uniform":
        b = make_uniform(T, spec["p"], spec["dim"], nq, seed, spec["pulse"])
    else:
        b = make_mixed(T, spec["choices"], spec["dim"], nq, seed, spec["pulse"])
    return b, spec


# ---------------------------------------------------------------- patches scattered in host memory
def scatter_to_host(batch: Batch, seed: int = 0) -> list:
    """The batch's patches as separate host arrays (one allocation each, made in a
    shuffled order so that consecutive patches do not sit side by side), as the
    patches of a mesh code live on the CPU heap.  Entry t is patch t."""
    rng = np.random.Generator(np.random.PCG64(seed))
    T = batch.num_patches
    order = rng.permutation(T)
    out = [None] * T
    for t in order:
        o = int(batch.offsets[t])
        n = int((int(batch.sizes[t]) + 2) ** batch.dim * batch.nq)
        out[t] = batch.data[o:o + n].copy()
    return out


# ---------------------------------------------------------------- states of the other PDEs
PDE_NAMES = ("euler", "shallow_water", "advection", "acoustics", "acoustics_ncp")
SWE_G = 9.81


def pde_unknowns(name: str, dim: int) -> int:
    """Unknowns per volume of a PDE (the layout the generator writes)."""
    return {"euler": 5, "shallow_water": 4, "advection": 1, "acoustics": 1 + dim, "acoustics_ncp": 1 + dim}[name]


def default_params(name: str) -> list:
    """Parameters of the synthetic workloads: gamma; g and the Coriolis parameter f; the
    advection velocity; rho0 and K0 of acoustics."""
    return {"euler": [GAMMA], "shallow_water": [SWE_G, 0.5], "advection": [0.7, -0.4, 0.25],
            "acoustics": [1.2, 2.0], "acoustics_ncp": [1.2, 2.0]}[name]


def make_pde_batch(name: str, sizes, dim: int = 2, seed: int = 0) -> Batch:
    """Contiguous batch of padded patches holding random states of the PDE `name`:
    Euler as make_batch; shallow water (h, hu, hv, b) with depth h in [1, 2], velocities in
    [-0.5, 0.5] and bathymetry b in [0, 0.3]; advection q in [-1, 1]; acoustics (p, u_1..u_d)
    in [-1, 1]."""
    sizes = np.asarray(sizes, dtype=np.int32)
    rng = np.random.Generator(np.random.PCG64(seed))
    if name == "euler":
        return make_batch(sizes, dim, 5, seed, rng=rng)
    nq = pde_unknowns(name, dim)
    nvol = int(np.sum((sizes.astype(np.int64) + 2) ** dim))
    if name == "shallow_water":
        if dim != 2:
            raise ValueError("shallow water is 2D")
        h = rng.uniform(1.0, 2.0, nvol)
        u = rng.uniform(-0.5, 0.5, nvol)
        v = rng.uniform(-0.5, 0.5, nvol)
        b = rng.uniform(0.0, 0.3, nvol)
        vols = np.stack([h, h * u, h * v, b], axis=1)
    else:
        vols = rng.uniform(-1.0, 1.0, (nvol, nq))
    return Batch(data=vols.reshape(-1).copy(), sizes=sizes, offsets=contiguous_offsets(sizes, dim, nq), dim=dim,
                 nq=nq)
