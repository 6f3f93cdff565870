"""CPU FP64 oracle for the Yin-Yang multipole gravity solve.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path imports this package:
only the test-suite, the smoke check and the CPU-baseline leg of the benchmark
may call it.  It shares no code with the HIP library; both sides receive their
inputs from the seeded workload generators, which hold none of the method's
arithmetic.

The oracle follows Almanstoetter, Melson, Janka & Mueller (2018), "Parallelized
solution method of the three-dimensional gravitational potential on the
Yin-Yang grid", equation by equation, in double precision.
"""

from .yyoracle import *  # noqa: F401,F403
