"""Seeded synthetic SPD matrices and job traces.

Input generation only: nothing here computes any step of the inversion method.
Both the GPU path and the CPU oracle consume these matrices; the matrix A is the
stored array itself (FP32 matrices are promoted exactly to FP64 by the oracle).

The paper's experiments (Sec. 10) use MATLAB `rand` matrices, LIBSVM ridge
Hessians (eq. ridgeMatrix) and SuiteSparse matrices; none of those datasets is
available here, so the families below stand in for them with the same structure:

  spectral_spd     A = Q diag(lambda) Q^T, Q from the QR of a Gaussian matrix,
                   lambda log-uniform; exact inverse Q diag(1/lambda) Q^T.
  gram_ridge       A = M^T M / n + mu I with Gaussian M (FP32).
  ridge_hessian    A = B^T B / m + lam I, B Gaussian m x n with columns scaled by
                   log-uniform factors (mimics heterogeneous feature scales of
                   the LIBSVM ridge Hessians of eq. ridgeMatrix), FP32.
  householder_spd  A = Q diag(lambda) Q^T with Q a product of r Householder
                   reflectors, formed in compact WY form (Q = I - V T V^T) so that
                   A = diag(lambda) + U C U^T is a rank-2r modification of a
                   diagonal matrix; exact inverse by the same construction.
  serving_trace    Poisson arrivals of jobs with log-uniform n.
"""
from .matrices import (spectral_spd, gram_ridge, ridge_hessian, ridge_data, householder_spd,
                       householder_factors, householder_entries, serving_trace,
                       CONFIGS)

__all__ = ["spectral_spd", "gram_ridge", "ridge_hessian", "ridge_data", "householder_spd",
           "householder_factors", "householder_entries", "serving_trace", "CONFIGS"]
