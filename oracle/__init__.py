"""FP64 CPU oracle of the raspberry / lattice-Boltzmann step.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the CPU-baseline leg of the
benchmark may import this package; the GPU library never does.  It shares no code with the
GPU library.  Build with ``python -m oracle.build`` (or ``oracle.build.build()``).
"""
