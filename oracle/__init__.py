"""FP64 CPU oracle for masked 4D Gaussian rasterization.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, links or runs
anything in this package; only the test suite, the smoke check and the
benchmark's CPU-baseline leg do.  It shares no code with the HIP library.

It states, plainly and slowly, what the renderer computes:

  slicing      Sec. 3, Eq. 1 (conditional 3D Gaussian) and Eq. 3 (temporal
               marginal p_i(t)) with Sigma = R S S^T R^T, R from (q_l, q_r)
  projection   local-affine (EWA) projection of the conditional Gaussian
  sh           view-dependent colour c_i(d), real SH up to degree 3
  composite    Eq. 2 / Eq. 3: per pixel, every Gaussian sorted by depth,
               front-to-back alpha blending (brute force, no tiles)
  mask         Sec. 4.2.2 keyframe active sets
  binning      the tile lists a tiled rasterizer must produce
  grad         torch float64 autograd of all of the above

Every function computes in float64.
"""
