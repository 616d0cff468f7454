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
    {1, 512, {8, 8, 16, 16, 16}},   // f64: 82.8 ms, 9.56 TFLOP/s; one launch per size class 91.3 ms
    {3, 256, {8, 16, 16, 16, 4}},   // f32: 62.7 ms, 12.61 TFLOP/s; one launch per size class 63.8 ms
    {3, 256, {8, 16, 16, 8, 16}},   // f32_bf16: 60.0 ms, 13.18 TFLOP/s; one launch per size class 63.4 ms
    {3, 256, {8, 16, 16, 16, 8}},   // f32_f16: 59.4 ms, 13.33 TFLOP/s; one launch per size class 62.3 ms
};

} // namespace stmg
