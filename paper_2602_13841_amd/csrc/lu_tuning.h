// Launch parameters of the persistent batched LU (stmg_batched_lu), per
// precision: workgroups per CU (which sets the LDS budget of the launch) and
// the panel width per size class.  Written by paper_2602_13841_amd/tune_lu.py
// (2026-12-03, AMD Radeon Graphics gfx950:sramecc+:xnack-) from the timings of the 4096-matrix mixed patch batch
// (sizes 85 ... 1185) noted beside each row.
#pragma once

namespace stmg {

constexpr int LU_TUNE_CLASSES = 5;
constexpr int LU_CLASS_MAX[LU_TUNE_CLASSES] = {128, 256, 512, 1024, 2048};

struct LuTune {
    int wg_per_cu;
    int threads;                 // per workgroup (one matrix): 256 or 512
    int nb[LU_TUNE_CLASSES];
};

// index: 0 = FP64, 1 = FP32, 2 = FP32 with BF16 update operands, 3 = FP16
constexpr LuTune LU_TUNED[4] = {
    {1, 512, {8, 8, 16, 16, 8}},   // f64: 77.9 ms, 10.16 TFLOP/s; one launch per size class 87.9 ms
    {3, 256, {8, 16, 16, 8, 4}},   // f32: 56.8 ms, 13.92 TFLOP/s; one launch per size class 63.6 ms
    {3, 256, {8, 16, 16, 8, 8}},   // f32_bf16: 53.1 ms, 14.89 TFLOP/s; one launch per size class 60.2 ms
    {3, 256, {8, 16, 16, 8, 16}},   // f32_f16: 52.9 ms, 14.96 TFLOP/s; one launch per size class 59.9 ms
};

} // namespace stmg
