"""FP64 CPU oracle of YAND-MVSK -- TEST INFRASTRUCTURE ONLY.

A plain, slow, deliberately unoptimised NumPy implementation of the method of
"Yau's Affine-Normal Descent for Large-Scale Unrestricted Higher-Moment
Portfolio Optimization" (Wang, Niu, Sheshmani, Yau).  It exists to check the
GPU library, never to serve it: only the tests, the smoke check and the CPU
baseline leg of the benchmark may import it.  It shares no code with the GPU
path; where the GPU works basis-free with projectors, this oracle builds the
explicit orthonormal bases the paper writes down (Section 4.2).
"""

from .mvsk import *  # noqa: F401,F403
