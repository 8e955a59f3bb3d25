"""Plain, slow, float64 CPU oracle of the articulated-body Stokes solver.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call,
link or execute anything in this package: only the tests, the smoke check and
the benchmark's CPU-baseline leg use it.  It shares no code with the GPU
library (``paper_2107_10800_amd``) and never reads values produced there.

Each function cites the passage of Balboa Usabiaga & Delmotte,
"A numerical method for suspensions of articulated bodies in viscous flows"
(arXiv:2107.10800) that it follows.  Readings of silent or garbled passages
are documented where they are taken.

Modules
  quat      unit quaternions and rotation matrices (Sec. 2.1, App. B)
  rpy       RPY blob mobility, unbounded and above a no-slip wall (Sec. 2.3)
  rpy_c     the same mobility as plain C loops (rpy_sum.c, OpenMP over targets;
            the wall image generated from rpy's symbolic definition by
            gen_wall_image_c.py): full products, dense matrices and solves at
            tens of thousands of blobs, and the timed CPU baseline
  bodies    blob positions, K, constraint Jacobian C and B (Sec. 2.2-2.3, App. A)
  system    the saddle system A y = b and its direct solutions (Sec. 2.2-2.3)
  precond   block-diagonal preconditioner (Sec. 3.1)
  gmres     right-preconditioned restarted GMRES (Sec. 3.1)
  correct   position/orientation correction (Sec. 4.2, App. B)
  timeloop  reconstruction of articulated bodies and the Euler step (Sec. 4.1, 4.3)
  rpy_rot   generalised RPY tensor of single-blob bodies, unbounded (Sec. 2.4)
  single_blob  the single-blob system Eq. linear_system_general and its preconditioner
  mlp       float64 MLP used to judge the learned body-mobility network
  fastsum   the interpolation-based multipole approximation of the blob
            mobility product (fast summation, Sec. 2.3 and Sec. 6)
"""
