"""The five benchmark workloads as seeded synthetic meshes.

Workload k uses seed ``CONFIG_SEED_BASE + k``:

1. 64-cell Voronoi of the unit square, 10 Lloyd iterations, p = 1.
2. 16,384-cell Voronoi (uniform seeds, no Lloyd), p = 2.
3. 262,144-cell Voronoi, per-cell p drawn uniformly from {1,2,3,4}.
4. 3D unit cube: 128^3 Kuhn tetrahedra agglomerated into 32,768 polyhedra, p = 2.
5. 262,144-cell Voronoi, p = 3.

Generated meshes are cached as ``.npz`` under ``$DGP_MESH_CACHE`` (default
``~/.cache/dgpoly-meshes``) keyed by their parameters.
"""

import hashlib
import os

import numpy as np

from .mesh import Mesh
from .voronoi import voronoi_mesh

CONFIG_SEED_BASE = 2007048810


def _cache_dir() -> str:
    d = os.environ.get("DGP_MESH_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "dgpoly-meshes"))
    os.makedirs(d, exist_ok=True)
    return d


def mesh_digest(mesh: Mesh) -> str:
    h = hashlib.sha256()
    for k in sorted(mesh.arrays()):
        a = np.ascontiguousarray(mesh.arrays()[k])
        h.update(k.encode())
        h.update(a.tobytes())
    return h.hexdigest()


def _save(path: str, mesh: Mesh) -> None:
    tmp = path + ".tmp.npz"
    np.savez(tmp, dim=mesh.dim, name=mesh.name, **mesh.arrays())
    os.replace(tmp, path)


def _load(path: str) -> Mesh:
    with np.load(path, allow_pickle=False) as z:
        d = {k: z[k] for k in z.files}
    dim = int(d.pop("dim"))
    name = str(d.pop("name"))
    return Mesh(dim=dim, name=name, **d)


GENERATOR_VERSION = "v2"


def cached(key: str, build) -> Mesh:
    path = os.path.join(_cache_dir(), f"{key}_{GENERATOR_VERSION}.npz")
    if os.path.exists(path):
        try:
            return _load(path)
        except Exception:
            os.remove(path)
    mesh = build()
    _save(path, mesh)
    return mesh


def config_mesh(k: int, n_cells: int = None) -> Mesh:
    """Mesh of workload ``k`` (1..5).  ``n_cells`` shrinks the 2D workloads for tests."""
    seed = CONFIG_SEED_BASE + k
    if k == 1:
        n = n_cells or 64
        return cached(f"cfg1_n{n}", lambda: voronoi_mesh(n, seed, lloyd=10, p=1))
    if k == 2:
        n = n_cells or 16384
        return cached(f"cfg2_n{n}", lambda: voronoi_mesh(n, seed, lloyd=0, p=2))
    if k == 3:
        n = n_cells or 262144

        def build():
            m = voronoi_mesh(n, seed, lloyd=0, p=1)
            rng = np.random.default_rng([seed, 1])
            return m.with_degrees(rng.integers(1, 5, size=m.n_cells).astype(np.int8))

        return cached(f"cfg3_n{n}", build)
    if k == 5:
        n = n_cells or 262144
        return cached(f"cfg5_n{n}", lambda: voronoi_mesh(n, seed, lloyd=0, p=3))
    if k == 4:
        from .kuhn import agglomerated_cube

        n = n_cells or 128
        return cached(f"cfg4_n{n}", lambda: agglomerated_cube(n, (n // 4) ** 3 if n >= 4 else 1, seed, p=2))
    raise ValueError(f"unknown workload {k}")


def problem_params(k: int) -> dict:
    """Coefficients and manufactured solution of workload ``k`` (plain data).

    a(x) = a0 + a1 sin(2 pi x) cos(2 pi y), b constant, c constant, penalty
    constant c_sigma; u = product of sines, with f and the Dirichlet data
    derived from it."""
    if k == 2:
        return dict(a0=1.0, a1=0.5, b=(1.0, 0.5, 0.0), c=1.0, c_sigma=10.0, u="sin")
    if k in (1, 3, 4, 5):
        return dict(a0=1.0, a1=0.0, b=(0.0, 0.0, 0.0), c=0.0, c_sigma=10.0, u="sin")
    raise ValueError(f"unknown workload {k}")
