"""Seeded synthetic bundle-adjustment problems.

This module only draws inputs: camera poses and intrinsics, landmark
positions, which cameras see which landmark, and the observed (distorted)
pixel of each observation under the undistortion camera model of Sec. III
(the ray [u/f; 1 + k1|u|^2 + k2|u|^4] is parallel to the point in the camera
frame).  It holds none of the method's arithmetic: no residual, no depth
scalar, no robust loss, no surrogate.  Both the CPU oracle and the GPU path
read the arrays it returns.
"""

from .problem import CONFIGS, make_problem, subproblem  # noqa: F401
