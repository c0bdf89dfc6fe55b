"""Seeded synthetic inputs shared by the oracle tests, the GPU tests and the
benchmark.  This module holds none of the factorisation's arithmetic: it only
draws matrices with a controlled singular spectrum.

Construction (the test matrices of Section 6.1 of Balabanov's paper: X =
U diag(sigma) V^T with orthonormal U, V and sigma_i = sigma_min^{i/(n-1)}):

* V (n x n) is the Q factor of an n x n Gaussian matrix with its column
  signs fixed so that diag(R) > 0 (Haar distributed; Mezzadri 2007).
* U (m x n) is the orthonormal polar factor G (G^T G)^{-1/2} of an m x n
  Gaussian matrix G.  The polar factor of a Gaussian matrix is Haar on the
  Stiefel manifold (left-orthogonal equivariance) and, unlike a tall
  Householder QR, needs only two streaming matrix products and an n x n
  symmetric eigendecomposition, so multi-GB inputs take seconds.
* X = G M with M = (G^T G)^{-1/2} diag(sigma) V^T, formed chunk by chunk.

FP32 inputs are the FP64 X rounded to nearest; the oracle then factors those
FP32 values promoted exactly to FP64.
"""
from .matrices import (spectrum, haar_square, make_x, make_x_torch,
                       make_cotangents, batched_shapes)

__all__ = ["spectrum", "haar_square", "make_x", "make_x_torch",
           "make_cotangents", "batched_shapes"]
