// Launchers of the comparison forms the library also offers: the sEnKF of
// Appendix A and the explicit-gain CGD-EnKF of Figure 2.
#pragma once

#include "internal.h"

namespace cgd {

// the sEnKF analysis (Appendix A) on the reduced mode's layout; iters0 (N
// ints, or NULL) receives zeros
template <typename T>
hipError_t launch_senkf(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                        const T* hw, const T* y, const T* rdiag, const T* eps, void* ws,
                        const Layout& L, int* iters0, hipStream_t s);

// Explicit-gain form (Figure 2): workspace offsets (bytes) and padded sizes;
// total 0 when the sizes or the precision are not supported (N > 128, not
// FP64 / FP32).
struct KtLayout {
  int NP, mp, nn;
  size_t S, D, rd, A, Z, R, P, status, iters, err, total;
};
KtLayout kt_layout(int n, int m, int N, int prec);
template <typename T>
hipError_t launch_kt(int n, int m, int N, int k, const T* Xf, T* Xa, const int32_t* idx,
                     const T* hw, const T* y, const T* rdiag, const T* eps, double tol, int maxit,
                     T* kt, int* iters, double* hist, const KtLayout& L, void* ws,
                     hipStream_t s);

}  // namespace cgd
