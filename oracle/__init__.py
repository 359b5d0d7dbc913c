"""CPU oracle -- TEST INFRASTRUCTURE ONLY.

A plain, slow, obviously correct implementation of what the GPU library
computes, used to check it.  Only the test suite, the smoke check and the
benchmark's CPU-baseline leg may import anything from here; the product
library never does, and nothing here imports the product library.

Contents
  native   -- ctypes wrapper over flux_oracle.c (binary64 flux, sequential
              edge loop, per-edge fluxes, first-fit colouring)
  exact    -- the same loop evaluated in exact rational arithmetic
  brute    -- cell-centric brute force residual for tiny meshes
  plans    -- integer-side checks: permutations, partitions, colourings,
              staged lists, reordering re-derivations
"""
