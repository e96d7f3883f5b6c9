"""MI355X (gfx950) randomized block BFGS matrix inversion.

Gower & Richtarik, "Randomized Quasi-Newton Updates are Linearly Convergent
Matrix Inversion Algorithms" (arXiv 1602.01768): fixed-sketch RBFGS (Sec. 8.7)
and AdaRBFGS (Sec. 9), behind the C ABI of include/rbfgs.h, with hand-written
HIP kernels in csrc/ and a ctypes binding in `rbfgs`.
"""
__all__ = ["rbfgs", "build"]
