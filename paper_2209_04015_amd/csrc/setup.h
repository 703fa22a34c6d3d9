// Internal launchers of the setup kernels (host-callable).
#pragma once

#include <hip/hip_runtime.h>

hipError_t setup_gemm(int M, int N, int K, int transA, const double* A, long lda, const double* B,
                      long ldb, double* C, long ldc, double* scratch, int nchunk, hipStream_t s);
hipError_t setup_hprime(int N, const double* h1, const double* LL, double* hp, double* tr,
                        hipStream_t s);
hipError_t setup_expm_arg(int N, const double* hp, double mu, double c, double* A, double* norm1,
                          hipStream_t s);
hipError_t setup_expm(int N, double* A, int sq, int order, double* R, double* T, hipStream_t s);
hipError_t setup_copy_pad(int rows, int cols, const double* src, int lds_, double* dst, int ldd,
                          hipStream_t s);
template <typename T>
hipError_t setup_pack_lh(int K, int N, int n, int nmax, int ldN, const double* Y, T* Lh,
                         hipStream_t s);
template <typename T>
hipError_t setup_pack_lt(int K, int N, int Npk, int ldK, const int2* pq, const double* L, T* LT,
                         hipStream_t s);
hipError_t setup_hh(int N, int n, int nmax, const double* phiT, const double* h1, double* hh,
                    hipStream_t s);
hipError_t setup_trial_walker(int N, int n, int nmax, const double* phiT, double2* phi,
                              hipStream_t s);
// rows (i, j >= i, p) over q of the pair integrals of one spin from C = Y^T Y
template <typename T>
hipError_t setup_pack_vpair(int N, int n, int Np, int ldq, long rows, const double* C, T* V, hipStream_t s);
