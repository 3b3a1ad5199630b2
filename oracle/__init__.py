"""Reference implementations used to check the GPU path.

TEST INFRASTRUCTURE ONLY.  Only tests/, __graft_entry__.smoke() and the CPU
baseline leg of bench.py may import anything here; the product package never
does, and shares no code with this package.

  ewald     - FP64 C direct Ewald sums (reciprocal energy/forces/virial,
              real-space and self terms for the Madelung check)
  ewald_np  - NumPy twin of the reciprocal sum for small systems
  pppm      - FP64 NumPy PPPM with ik-differentiation (full spectra)
  learned   - FP64 NumPy descriptor, MLP, force head, manual backprop and Adam
              of the learned coarse-mesh correction
"""
