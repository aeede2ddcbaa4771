// Library primitives used by the pair bucketing: stable radix sort of int32
// key/value pairs and exclusive prefix sums (rocPRIM).
#include <cstring>
#include <rocprim/device/device_radix_sort.hpp>
#include <rocprim/device/device_scan.hpp>
#include <rocprim/iterator/transform_iterator.hpp>

#include "pgx_prim.hpp"

namespace pgx {

namespace {
struct U8ToInt {
  __host__ __device__ int32_t operator()(uint8_t v) const { return (int32_t)v; }
};
}  // namespace

void sort_pairs_i32(const int32_t* kin, int32_t* kout, const int32_t* vin, int32_t* vout, int64_t n,
                    int end_bit, hipStream_t s, DBuf& tmp) {
  if (n <= 0) return;
  size_t bytes = 0;
  PGX_HIP(rocprim::radix_sort_pairs(nullptr, bytes, kin, kout, vin, vout, (size_t)n, 0, end_bit, s));
  void* t = tmp.ensure(bytes);
  PGX_HIP(rocprim::radix_sort_pairs(t, bytes, kin, kout, vin, vout, (size_t)n, 0, end_bit, s));
}

void exscan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s, DBuf& tmp) {
  if (n <= 0) return;
  size_t bytes = 0;
  PGX_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, (int64_t)0, (size_t)n,
                                  rocprim::plus<int64_t>(), s));
  void* t = tmp.ensure(bytes);
  PGX_HIP(rocprim::exclusive_scan(t, bytes, in, out, (int64_t)0, (size_t)n, rocprim::plus<int64_t>(), s));
}

void exscan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s, DBuf& tmp) {
  if (n <= 0) return;
  size_t bytes = 0;
  PGX_HIP(rocprim::exclusive_scan(nullptr, bytes, in, out, (int32_t)0, (size_t)n,
                                  rocprim::plus<int32_t>(), s));
  void* t = tmp.ensure(bytes);
  PGX_HIP(rocprim::exclusive_scan(t, bytes, in, out, (int32_t)0, (size_t)n, rocprim::plus<int32_t>(), s));
}

void exscan_u8_i32(const uint8_t* in, int32_t* out, int64_t n, hipStream_t s, DBuf& tmp) {
  if (n <= 0) return;
  auto it = rocprim::make_transform_iterator(in, U8ToInt());
  size_t bytes = 0;
  PGX_HIP(rocprim::exclusive_scan(nullptr, bytes, it, out, (int32_t)0, (size_t)n,
                                  rocprim::plus<int32_t>(), s));
  void* t = tmp.ensure(bytes);
  PGX_HIP(rocprim::exclusive_scan(t, bytes, it, out, (int32_t)0, (size_t)n, rocprim::plus<int32_t>(), s));
}

}  // namespace pgx
