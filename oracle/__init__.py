"""CPU oracle for the SQD hot path -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library never does, and
this package never imports the product: the two share only the seeded input
generators of ``paper_2601_16169_amd.inputs``.

Modules:
  core      -- ctypes front end of the plain C oracle (sqd_oracle.c):
               sigma, per-term sigma, sampled rows, diagonal, dense H, RDMs.
  davidson  -- textbook Davidson-Liu (lowest root) over the oracle sigma,
               plus the dense-eigh route for small spaces.
  tables    -- per-string single/double excitation lists built with Python
               sets and dicts, signs from explicit operator application.
  fock      -- Jordan-Wigner brute force on the full Fock space (norb <= 5),
               the pin for signs and matrix elements.
"""
