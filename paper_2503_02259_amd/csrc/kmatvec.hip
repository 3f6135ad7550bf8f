// Dispatch of the on-the-fly kernel MatVec to its precision forms.
#include <atomic>

#include "common.h"

namespace higp {

int launch_kmatvec_f32(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                       int num_cus);
int launch_kmatvec_f64(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                       int num_cus);
int launch_kmatvec_bf16(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                        int num_cus, bool split);
int launch_kmatvec_f32_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                             void* Y, hipStream_t st, int num_cus);
int launch_kmatvec_f64_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                             void* Y, hipStream_t st, int num_cus);

namespace {

int num_cus_impl() {
  static std::atomic<int> cached[64];  // per device; 0 = not yet queried
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int cus = cached[dev].load(std::memory_order_relaxed);
  if (cus == 0) {
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev].store(cus, std::memory_order_relaxed);
  }
  return cus;
}

int num_cus() { return num_cus_impl(); }

}  // namespace

int device_num_cus() { return num_cus_impl(); }

int launch_kmatvec(const Problem& p, int k, const void* V, MatvecOut out, hipStream_t st,
                   int prec_override) {
  const int prec = prec_override >= 0 ? prec_override : p.prec;
  if (prec == HIGP_FP64) return launch_kmatvec_f64(p, k, V, out, st, num_cus());
  if (prec == HIGP_FP32) return launch_kmatvec_f32(p, k, V, out, st, num_cus());
  if (prec == HIGP_BF16) return launch_kmatvec_bf16(p, k, V, out, st, num_cus(), false);
  if (prec == HIGP_BF16X3) return launch_kmatvec_bf16(p, k, V, out, st, num_cus(), true);
  return set_error(HIGP_ERR_UNSUPPORTED, "precision %d is not implemented for this MatVec", prec);
}

int launch_kmatvec_cross(const Problem& p, int64_t m, const void* Xq, int k, const void* V,
                         void* Y, hipStream_t st) {
  if (p.prec == HIGP_FP64) return launch_kmatvec_f64_cross(p, m, Xq, k, V, Y, st, num_cus());
  if (p.prec == HIGP_FP32) return launch_kmatvec_f32_cross(p, m, Xq, k, V, Y, st, num_cus());
  return set_error(HIGP_ERR_UNSUPPORTED, "the rectangular MatVec runs in FP64 or FP32");
}

}  // namespace higp
