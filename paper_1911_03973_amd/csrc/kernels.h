// kernels.h -- launchers of the device kernels (internal to libfem).
#pragma once

#include <hip/hip_runtime.h>

#include "plan.h"

namespace fem {

// Default workgroup size of the solver's element pass for a chunk size.
int default_block(int nb, int E);
int device_cu_count();

int launch_local_matrices(const DevPlan &P, int kind, void *K, void *M, double *vol, hipStream_t s);
int launch_combine(const DevPlan &P, int kin, const void *K, const void *M, double nu, int kout, void *A,
                   hipStream_t s);

// out = (b ? b : 0) + sign * sum_e C_e^T A_e C_e x, optionally masked (out(nd) = 0).
// scratch: n_partials doubles.
int launch_apply64(const DevPlan &P, int kind, const void *K, const void *M, double nu, const double *x,
                   const double *b, double *out, double sign, int use_mask, double *scratch, hipStream_t s);
// the same with float matrices, vectors and accumulation; scratch: n_partials floats
int launch_apply32(const DevPlan &P, const float *A, const float *x, const float *b, float *out, float sign,
                   int use_mask, float *scratch, hipStream_t s);
// The same through the packed difference form (kind MAT_F64 or MAT_F32X2).
int launch_apply_pk64(const DevPlan &P, int kind, const void *A, const double *x, const double *b, double *out,
                      double sign, int use_mask, double *scratch, hipStream_t s);
// Packed difference form of A_e = K_e + nu M_e (FP64 arithmetic), stored as
// kout = MAT_F64 or MAT_F32X2.
int launch_pack(const DevPlan &P, int kin, const void *K, const void *M, double nu, int kout, void *A,
                hipStream_t s);
// d = sum_e C_e^T diag(A_e) from the packed difference form
int launch_diag_pk64(const DevPlan &P, int kind, const void *A, double *d, double *scratch, hipStream_t s);
// Matrix-free (K_e, M_e rebuilt from the plan's coordinates in every pass):
// out = (b ? b : 0) + sign * sum_e C_e^T (kk K_e + nu M_e) C_e x, and the
// diagonal of K + nu M.  FEM_EINVAL when the chunk's LDS exceeds the limit.
int launch_apply_mf(const DevPlan &P, double kk, double nu, const double *x, const double *b, double *out,
                    double sign, int use_mask, double *scratch, hipStream_t s);
int launch_diag_mf(const DevPlan &P, double nu, double *d, double *scratch, hipStream_t s);
// Dynamic LDS one workgroup may use on the current device.
size_t device_lds_limit();
// d = sum_e C_e^T diag(A_e)
int launch_diag64(const DevPlan &P, int kind, const void *K, const void *M, double nu, double *d,
                  double *scratch, hipStream_t s);

}  // namespace fem
