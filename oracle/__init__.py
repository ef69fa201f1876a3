"""FP64 CPU oracle for path collective variables with a floating close structure.

TEST INFRASTRUCTURE ONLY.  Nothing in the library imports this package; it
exists so that tests, the smoke check and the CPU-baseline leg of the
benchmark can check the HIP path against a plain, slow, obviously correct
implementation written from the paper (arXiv:1801.02362):

* ``oracle.msd``   -- O1: Eq. 3 (exact MSD after optimal superposition) and
  Eq. 4 (its derivative), with the rotation from the top eigenpair of the
  4x4 quaternion matrix (Section 3, the Kearsley / Coutsias construction).
* ``oracle.path``  -- O2: Eq. 2 (property-map CV, ``q_i = i`` gives the path
  variable ``s``) and the path distance ``z``; gradients by the chain rule.
* ``oracle.close`` -- O3: Algorithm 2 (floating close structure), Eq. 5 and
  Eq. 6, including the derivative of the close-structure rotation.
* ``oracle.cost``  -- O4: the cost model of Section 6.2 and Eq. 7.
* ``oracle.mlp``   -- O5: FP64 reference of the surrogate network.
* ``oracle.bias``  -- O6: the metadynamics bias of Eq. 1 on (s, z), kept on
  a grid with bicubic Hermite interpolation, and its gradient on the atoms.
* ``oracle.nl``    -- O7: neighbour lists (Section 2) with Algorithm 1 and
  with the close structure (selection by Eq. 5 at list updates, Section 3.2).
* ``oracle.props`` -- O8: property maps with several properties per
  reference (Eq. 2 with a vector q_i).

Everything is FP64 NumPy on FP64 copies of the caller's (possibly FP32)
inputs.  The oracle shares no code, header, table or constant with the HIP
path.  Pins (tests marked ``not gpu``) tie each function to facts that do not
come from the oracle itself: rigid-copy and symmetry invariants, brute force
over a rotation grid, an SVD-based superposition, the roots of the
characteristic polynomial, central finite differences, closed forms of the
path variables and the paper's own cost arithmetic.

Parity unpinned: the size of the close-structure approximation error on the
synthetic random walk and the number of reassignments it needs (the paper's
values are for real MD trajectories); the surrogate network's accuracy.
"""
