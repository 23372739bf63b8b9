"""FP64 CPU oracle for the BiP-PRISM core-loss STEM-EELS hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports, calls or
links anything under this directory; only the tests, the smoke check and the
benchmark's CPU-baseline leg do.  The oracle shares no code with the HIP
library: it is a plain, slow, float64/complex128 restatement of the paper's
forward model and algorithms, using numpy/scipy FFTs and matrix products as
library primitives, written so that each step can be checked against the
paper by eye.

Modules
  physics    -- wavelength, interaction constant, beam sets, operators
  sibson     -- natural-neighbour (Sibson) weights on the parent lattice
  multislice -- multislice step, its transpose, parent-column sweeps
  eels       -- Alg. 1 (conventional), Alg. 4 (exact dual matrix),
                Alg. 5 (BiP-PRISM), windowed reconstruction, contraction,
                output reductions, on-atom diagnostic
  adjoint    -- gradient of a map loss through Alg. 5 (slice potentials,
                transition potentials, atom positions)
  potential  -- slice potentials from atom positions and their gradient
"""
