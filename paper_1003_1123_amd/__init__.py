"""On-the-fly random numbers for Langevin dynamics on AMD MI355X (gfx950).

Zhmurov, Rybnikov, Kholodov & Barsegov, arXiv:1003.1123: Hybrid Taus and Ran2 (one generator per
thread) and additive lagged Fibonacci (one generator for all threads), Box-Muller, and a fused
Langevin-dynamics update of independent 3-D harmonic oscillators.  The compute path is librngld.so
(hand-written HIP, C ABI in include/rngld.h); `_lib` binds it and `autograd` wraps the adjoint.
"""
