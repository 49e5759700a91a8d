"""Seeded synthetic input generators shared by the tests, the benchmark and the oracle.

This package holds no arithmetic of the method: it only produces meshes (element
vertex coordinates), initial velocity fields and seeded random data.  Both the
CPU oracle (``oracle/``) and the GPU library consume what it produces; neither
side's computations live here.
"""
from .meshes import (periodic_split_square, channel_split_square, distort_split_square, element_order,  # noqa: F401
                     inout_split_square, outflow_at_right, periodic_kuhn_cube, channel_kuhn_cube,
                     inout_kuhn_cube)
from .fields import (  # noqa: F401
    taylor_green_2d,
    channel_shear_layer,
    double_shear_layer,
    RandomStreamField,
    random_broken_poly,
    eval_broken_poly,
    n_monomials,
    taylor_green_3d,
    abc_flow,
    RandomVectorPotentialField,
    random_broken_poly_3d,
    eval_broken_poly_3d,
    n_monomials_3d,
)
