// Opt-in per-kernel timing with HIP events recorded on the launch stream.
// Disabled by default; when disabled a scope costs one branch.
#pragma once

#include <hip/hip_runtime.h>

namespace gs {

enum KernelId {
    K_FFT_ROWS_T = 0, K_FFT_COLS_T, K_FFT_SIDECOLS_T, K_INTERP2D, K_INTERP1D, K_FFT1_T,
    K_ADJ_PREP, K_BOUNDARY_PARTIAL, K_BOUNDARY_FINAL, K_SPREAD2D, K_SIDE_ROWS, K_SIDE_COLS, K_REDUCE_STRIPS,
    K_FFT_COLS_TH, K_FFT_ROWS_TH, K_FFT_SIDECOLS_TH, K_SPREAD1D, K_FFT1_TH, K_MERGE, K_BND2D, K_INTERP_BND,
    K_CNN_FIRST, K_CNN_CONV, K_CNN_LAST, K_CNN_LOSS, K_CNN_LAST_BWD, K_CNN_CONV_BWD, K_CNN_DW, K_CNN_DW_THIN,
    K_CNN_STEP, K_COUNT
};

extern bool g_prof_enabled;
void prof_record(int id, hipStream_t s, bool begin);

struct ProfScope {
    int id;
    hipStream_t s;
    ProfScope(int i, hipStream_t st) : id(i), s(st) {
        if (g_prof_enabled) prof_record(id, s, true);
    }
    ~ProfScope() {
        if (g_prof_enabled) prof_record(id, s, false);
    }
};

}  // namespace gs
