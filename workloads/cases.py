"""Named synthetic workloads (mesh recipe + H2 parameters + right-hand sides).

Each case stands in for one of the paper's test geometries (Section 5: sphere,
flat prism, torus), whose tetrahedral meshes are not available; sizes follow
the paper's regime of 10^5..10^6 boundary nodes (Section 6.1).
"""
from __future__ import annotations

from dataclasses import dataclass, field

from . import meshes

__all__ = ["MeshSpec", "Case", "CASES", "mesh_of", "SERVING_MESHES"]


@dataclass(frozen=True)
class MeshSpec:
    kind: str                 # "icosphere" | "cuboid" | "torus"
    level: int = 0            # icosphere subdivision level
    jitter: float = 0.0       # icosphere: relative radial; cuboid: absolute in-plane (nm)
    seed: int = 0

    @property
    def name(self) -> str:
        if self.kind == "icosphere":
            return f"sphere_l{self.level}"
        return self.kind


@dataclass(frozen=True)
class Case:
    name: str
    mesh: MeshSpec
    order: int
    leaf: int
    eta: float
    nrhs: int
    precisions: tuple = ("fp64",)
    notes: str = ""


def mesh_of(spec: MeshSpec):
    if spec.kind == "icosphere":
        return meshes.icosphere(spec.level, spec.jitter, spec.seed)
    if spec.kind == "cuboid":
        return meshes.cuboid(2000.0, 2000.0, 20.0, 5.0, spec.jitter, spec.seed)
    if spec.kind == "torus":
        return meshes.torus(1.0, 0.3, 256, 64)
    raise ValueError(spec.kind)


SPHERE_L4 = MeshSpec("icosphere", 4, 0.01, 0)
SPHERE_L5 = MeshSpec("icosphere", 5, 0.01, 0)
SPHERE_L6 = MeshSpec("icosphere", 6, 0.005, 0)
SPHERE_L7 = MeshSpec("icosphere", 7, 0.005, 0)
SPHERE_L8 = MeshSpec("icosphere", 8, 0.0025, 0)
FILM = MeshSpec("cuboid", 0, 0.5, 0)
TORUS = MeshSpec("torus")

CASES = {
    # 2562 nodes: small enough for the dense matrix and the full H2 oracle
    "sphere_l4": Case("sphere_l4", SPHERE_L4, 4, 32, 2.0, 2, ("fp64",),
                      "u1 = z and u1 ~ N(0,1) (seed 0)"),
    # 163842 nodes: FP64 against FP32, u1 = z plus 8 N(0,1) columns
    "sphere_l7": Case("sphere_l7", SPHERE_L7, 4, 64, 2.0, 9, ("fp64", "fp32")),
    # thin film 2000 x 2000 x 20 nm on a 5 nm grid, 326402 nodes
    "film": Case("film", FILM, 5, 64, 2.0, 4, ("fp32",)),
    # 655362 nodes, 16 RHS: the largest single-GPU case
    "sphere_l8": Case("sphere_l8", SPHERE_L8, 5, 64, 2.0, 16, ("fp32", "bf16x3", "fp64")),
}

# resident meshes of the serving mix: (spec, order, leaf)
SERVING_MESHES = [
    (SPHERE_L4, 4, 64), (SPHERE_L5, 4, 64), (SPHERE_L6, 4, 64), (SPHERE_L7, 4, 64),
    (FILM, 5, 64), (TORUS, 4, 64),
]
