// Nyström preconditioner (farthest-point landmarks, Woodbury apply); see
// nystrom.hip.
#pragma once

#include "common.h"

namespace higp {

struct NysPrec {
  void* mem = nullptr;     // one stream-ordered allocation holding everything below
  int64_t n = 0;
  int r = 0, kmax = 0, prec = 0, S = 1;
  int64_t chunk = 0;       // rows per partial-sum chunk of WᵀR
  double s = 0.0;
  void* W = nullptr;       // n×r, element type of the problem
  double* Cinv = nullptr;  // r×r
  int* sel = nullptr;      // r landmark indices
  double* part = nullptr;  // S×r×kmax
  double* Tm = nullptr;    // r×kmax
  double* u = nullptr;     // r×kmax
};

// Build for problem p (s > 0) with `rank` landmarks (clamped to n) and
// right-hand-side blocks up to kmax columns.  Synchronises `st`.
int nys_build(const Problem& p, int rank, int kmax, NysPrec* P, hipStream_t st);
// Z = M⁻¹R for an n×k FP64 block (k ≤ kmax); asynchronous.
int nys_apply(const NysPrec& P, int k, const double* R, double* Z, hipStream_t st);
void nys_free(NysPrec& P, hipStream_t st);
// Device bytes a built preconditioner holds (kept until nys_free).
size_t nys_bytes(int64_t n, int rank, int kmax, int prec);
// The min(rank, n) farthest-point landmarks into host memory; synchronises.
int fps_landmarks(const Problem& p, int rank, int* sel_host, hipStream_t st);

}  // namespace higp
