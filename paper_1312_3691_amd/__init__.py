"""MI355X-native test-particle Monte Carlo (TPMC) free-molecular drag.

Hot path (Parham & Barba, "Finding the Force"): seed test particles on a
spherical control volume with the flux-correct drifting-Maxwellian
distribution (Sec. III.A), ray-trace them through a triangulated body with
specular / diffuse re-emission (Sec. II.A), and sum the momentum they give each
triangle into force, moment and drag coefficient (eq. drag).

``paper_1312_3691_amd.tpmc`` is the Python binding of the C-ABI library
``libtpmc.so`` (HIP kernels for gfx950); importing it fails loudly when the
library has not been built.  ``paper_1312_3691_amd.inputs`` builds synthetic
meshes and query records.
"""

__all__ = ["inputs"]
