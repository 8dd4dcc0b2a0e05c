"""FP64 CPU oracle for the regularized-Brinkmanlet filament swimmer and the
ABC / surrogate machinery around it.

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import, call or load anything here.  The
product package never imports it, and the two share no code: the only shared
module is the seeded input generator, which holds none of the method's
arithmetic.

Layout
  swim_oracle.c  -- kernel (eq. BrV with the blob reading), forces (EFB, curva,
                    EFT), forward-Euler runs; plain loops, FP64 state,
                    extended-precision kernel values.
  build.py       -- compiles swim_oracle.c with gcc into liboracle.so.
  core.py        -- ctypes wrappers around liboracle.so.
  abc.py         -- ABC distance, percentile tolerance, PMC weights and
                    proposal generation (numpy, FP64).
  philox.py      -- Philox4x32-10 counter-based generator (Salmon et al. 2011).
  mlp.py         -- FP64 surrogate MLP forward/backward, GELU, Adam.
"""
