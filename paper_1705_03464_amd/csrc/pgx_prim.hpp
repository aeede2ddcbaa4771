#pragma once
#include "pgx_host.hpp"

namespace pgx {
void sort_pairs_i32(const int32_t* kin, int32_t* kout, const int32_t* vin, int32_t* vout, int64_t n,
                    int end_bit, hipStream_t s, DBuf& tmp);
void exscan_i64(const int64_t* in, int64_t* out, int64_t n, hipStream_t s, DBuf& tmp);
void exscan_i32(const int32_t* in, int32_t* out, int64_t n, hipStream_t s, DBuf& tmp);
void exscan_u8_i32(const uint8_t* in, int32_t* out, int64_t n, hipStream_t s, DBuf& tmp);
}  // namespace pgx
