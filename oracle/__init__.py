"""CPU oracle for the SBR trace-integrate path.

TEST INFRASTRUCTURE ONLY.  This package is the slow, obviously-correct
reference against which the HIP path is checked.  It may be imported only by
``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py``; the product package never imports it and shares no code with
it (inputs come from the separate ``sbr_inputs`` generators).

Parity status per function (pins are in ``tests/test_oracle_*.py``):
  frame, aperture, gen_rays  pinned (ray counts of Eq. L3 by hand, frame
                             orthonormality, grid spacing/centring)
  trace (brute force)        pinned (hand-computed tiny meshes, plate and
                             trihedral/dihedral geometry, invariants)
  trace (BVH fast mode)      pinned to brute force, bit-exact
  po (PAPER, VECTOR)         pinned (plate closed form, trihedral peak,
                             dihedral polarimetric sign, translation phase)
  mie                        pinned (Rayleigh and optical limits)
  mlp (surrogate network)    pinned (finite differences of the float64
                             network, bf16 rounding cases, hand-written
                             special cases, Adam first-step property)
"""
