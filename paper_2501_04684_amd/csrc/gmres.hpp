// Restarted GMRES for (sigma I + Z^F) x = b on one plan: device state and
// the kernel launchers (gmres.hip). All sums, norms and the Hessenberg /
// Givens / least-squares state are FP64; Krylov vectors are complex64.
#pragma once

#include <hip/hip_runtime_api.h>
#include <hip/hip_vector_types.h>

#include <cstdint>

namespace ubf {

constexpr int kMaxRestart = 128;  // Krylov columns per cycle (restart length)
constexpr int kMaxGmresRhs = 64;  // right-hand sides per solver
constexpr int kDotBlocks = 256;   // fixed block count of the two-level sums

// Per-RHS row copied to the host after each step.
struct GmresStatusRow {
  double res;     // relative residual estimate |g_{k}| / ||b||
  int32_t active; // 1 while the right-hand side is still iterating
  int32_t iters;  // Arnoldi steps taken
};

// Device pointers into the solver workspace (passed to kernels by value).
struct GmresState {
  int m;            // restart length
  double2* H;       // [R][m][m+1]: column j of rhs r at (r*m + j)*(m+1)
  double2* h1;      // [R][m+1] first Gram-Schmidt pass
  double2* h2;      // [R][m+1] second pass
  double2* nrm;     // [R] sum |w|^2 (real part)
  double* cs;       // [R][m] Givens cosines
  double2* sn;      // [R][m] Givens sines
  double2* g;       // [R][m+1] rotated least-squares right-hand side
  double2* y;       // [R][m] cycle coefficients
  double* scale;    // [R] 1 / h_{j+1,j} (0 when inactive)
  double* bnorm;    // [R] ||b||
  double* res;      // [R] relative residual estimate
  int32_t* active;  // [R]
  int32_t* k;       // [R] columns of the current cycle
  int32_t* iters;   // [R]
};

int gmres_dot_blocks(int64_t n);
int launch_gmres_dots(const float2* V, int64_t vstride, int ncol, const float2* w, int64_t n,
                      int R, double2* partial, double2* out, int ldo, hipStream_t s);
int launch_gmres_update(const float2* V, int64_t vstride, int ncol, const double2* h, int ldh,
                        float2* w, int64_t n, int R, hipStream_t s);
int launch_gmres_add_shift(float2* w, const float2* v, double sr, double si, int64_t total,
                           hipStream_t s);
int launch_gmres_scale(float2* dst, const float2* src, const double* sc, int64_t n, int R,
                       hipStream_t s);
int launch_gmres_residual(float2* dst, const float2* b, const float2* x, const float2* ax,
                          double sr, double si, int64_t total, hipStream_t s);
int launch_gmres_cycle_start(const GmresState& st, int R, int first, double tol, hipStream_t s);
int launch_gmres_tail(const GmresState& st, int R, int j, double tol, hipStream_t s);
int launch_gmres_backsolve(const GmresState& st, int R, hipStream_t s);
int launch_gmres_combine(const float2* V, int64_t vstride, const GmresState& st, float2* x,
                         int64_t n, int R, hipStream_t s);
int launch_gmres_status(const GmresState& st, int R, GmresStatusRow* out, hipStream_t s);
int launch_gmres_zero(float2* p, int64_t total, hipStream_t s);
int launch_gmres_rand(float2* v, int64_t n, uint64_t seed, hipStream_t s);
int launch_gmres_conj(float2* dst, const float2* src, int64_t n, hipStream_t s);
int launch_gmres_inv_norm(const double2* nrm, double* scale, hipStream_t s);

}  // namespace ubf
