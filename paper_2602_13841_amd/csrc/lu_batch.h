// Standalone batched LU driver (internal).
#pragma once

#include "../../include/stmg.h"

#include <hip/hip_runtime.h>
#include <stddef.h>

namespace stmg {

struct LuTune;

// where the per-matrix metadata the kernels read is staged: a per-call device
// allocation, or the library's fixed per-device array (no allocation)
enum class MetaStaging { PerCall, Fixed };

size_t batched_lu_meta_bytes(int batch);

// factorization (solve == false) or substitution (solve == true) of a batch
// of matrices of mixed sizes; argument meaning as in stmg_batched_lu and
// stmg_batched_lu_solve; cfg: launch parameters (NULL = the tuned table);
// returns an STMG_ code and synchronizes the stream
int batched_lu_run(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                   const long long *p_off, int *info, void *b, const long long *b_off, void *stream, bool solve,
                   MetaStaging staging, const LuTune *cfg = nullptr);

} // namespace stmg
