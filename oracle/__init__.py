"""Plain, slow FP64 CPU oracle for the RBF-FD surface method.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and
the ``cpu_baseline`` leg of ``bench.py`` may import anything from here.  The
HIP library and its Python binding never import it, and it imports nothing
from them: the two share no code, constants or helpers.  Inputs come from
the ``synth`` package, which holds no arithmetic of the method.

Modules:
  knn      -- stencil membership (Sec. 4: centre plus its n-1 nearest
              neighbours by Euclidean distance in R^3).
  weights  -- radial kernels, the local RBF interpolation system, projected
              gradient matrices B^d, G^d = B^d A^{-1}, L_P = sum_d G^d G^d and
              the first-row weights (Secs. 2-4, eqs. srbfinterp, rbf_linsys,
              proj_mat, grad, Lap, surface_lap_P1).
  shape    -- condition number kappa_2 and the per-stencil shape parameter
              search to a target condition number (Sec. 5, eq. target_cond).
  stepper  -- sparse L_X and the method-of-lines right-hand side with RK4
              (Sec. 4.2, eq. kernel_mol).
  mlp      -- FP64 forward/backward of the shape-parameter regressor.
  truth    -- 60-digit mpmath weights for small stencils.
"""
