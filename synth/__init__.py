"""Seeded synthetic inputs shared by the CPU oracle and the HIP path.

This package generates meshes, boundary data, material parameter sets and
random vectors.  It holds none of the method's arithmetic (no residual, no
tangent, no solver step): every number it produces is problem data that both
sides consume independently.
"""
from .mesh import (cube_mesh, tube_mesh, strip_mesh, strip_dims, helical_fibres, planar_fibres,
                   fibre_field, Mesh)
from .cases import (Material, TimeInt, cube_case, tube_case, strip_case, material_from_nu,
                    random_vector, random_state, NH_COMP, NH_INCOMP, HGO_INCOMP)

__all__ = ["cube_mesh", "tube_mesh", "strip_mesh", "Mesh", "Material", "TimeInt",
           "cube_case", "tube_case", "strip_case", "material_from_nu", "fibre_field"]
