// Host real Schur decomposition (see schur_host.cpp).
#pragma once

namespace lyap {

// A = Z T Z^T with Z orthogonal and T quasi-upper-triangular (1x1 blocks and
// 2x2 blocks holding complex-conjugate pairs).  Row-major n x n in and out.
// Returns false if the QR iteration did not converge.
bool real_schur(int n, const double* A_rowmajor, double* T_rowmajor, double* Z_rowmajor,
                int* iterations);

}  // namespace lyap
