// Standalone batched LU factorizations and solves of mixed-size dense
// matrices (the Vanka patch factorization of Sec. "Inexact space-time Vanka
// smoother" as a batch of its own): host driver shared by stmg_batched_lu,
// stmg_batched_lu_solve and the allocation-free stmg_batched_lu_noalloc.
//
// The per-matrix metadata (size, element offset of the matrix, of its pivots
// and of its right-hand side, sorted by decreasing size) is staged in device
// memory for the kernels: in a per-call allocation, or, for callers that
// cannot allocate, in the file-scope array `scratch` below.
#include "lu_batch.h"
#include "lu_tuning.h"
#include "vanka.h"

#include <algorithm>
#include <cstring>
#include <mutex>
#include <vector>

namespace stmg {

namespace {

// metadata of one matrix: m and the panel width (two ints in one 8-byte
// slot), a_off, p_off, b_off; plus one 256-byte slot for the queue counter
constexpr size_t META_BYTES_PER_MATRIX = 4 * sizeof(long long);
constexpr size_t META_HEADER_BYTES = 256;

// the fixed staging of the allocation-free entry point, one copy per device
// (each device that runs the library keeps it until the process ends)
constexpr size_t SCRATCH_BYTES = (size_t)STMG_NOALLOC_MAX_BATCH * META_BYTES_PER_MATRIX + META_HEADER_BYTES;
static __device__ __align__(256) unsigned char scratch[SCRATCH_BYTES];

constexpr int MAX_DEVICES = 64;

// device address of `scratch` on the current device, looked up once per
// device (host code must not use the symbol's name as an address)
int scratch_address(void **out)
{
    static std::mutex mu;
    static void *addr[MAX_DEVICES] = {nullptr};
    int dev = 0;
    if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= MAX_DEVICES) return STMG_EHIP;
    std::lock_guard<std::mutex> lk(mu);
    if (!addr[dev]) {
        void *p = nullptr;
        if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) {
            (void)hipGetLastError();
            return STMG_EHIP;
        }
        addr[dev] = p;
    }
    *out = addr[dev];
    return STMG_OK;
}

struct DevAlloc {
    void *p = nullptr;
    ~DevAlloc()
    {
        if (p) (void)hipFree(p);
    }
};

} // namespace

size_t batched_lu_meta_bytes(int batch) { return META_HEADER_BYTES + (size_t)batch * META_BYTES_PER_MATRIX; }

namespace {

int tune_index(int prec)
{
    return prec == STMG_F64 ? 0 : prec == STMG_F32 ? 1 : prec == STMG_F32_BF16 ? 2 : 3;
}

int size_class(int m)
{
    int c = 0;
    while (c + 1 < LU_TUNE_CLASSES && m > LU_CLASS_MAX[c]) ++c;
    return c;
}

int device_cus()
{
    int dev = 0, n = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        n < 1)
        n = 256;
    return n;
}

} // namespace

int batched_lu_run(int prec, void *A, const long long *a_off, const int *m_of, int batch, int *piv,
                   const long long *p_off, int *info, void *b, const long long *b_off, void *stream, bool solve,
                   MetaStaging staging, const LuTune *cfg)
{
    if (!A || !a_off || !m_of || !piv || !p_off || batch < 0) return STMG_EINVAL;
    if (prec != STMG_F64 && prec != STMG_F32 && prec != STMG_F32_BF16 && prec != STMG_F32_F16) return STMG_EINVAL;
    if (solve && (!b || !b_off)) return STMG_EINVAL;
    if (staging == MetaStaging::Fixed && batch > STMG_NOALLOC_MAX_BATCH) return STMG_EINVAL;
    if (batch == 0) return STMG_OK;
    // FP32 storage for the three FP32 variants; op = operands of the
    // trailing-update MFMA
    const int op = prec == STMG_F32_BF16 ? 1 : (prec == STMG_F32_F16 ? 2 : 0);
    std::vector<int> ord(batch);
    int maxm = 0;
    for (int i = 0; i < batch; ++i) {
        ord[i] = i;
        if (m_of[i] < 1 || m_of[i] > 2048 || a_off[i] < 0 || p_off[i] < 0 || (solve && b_off[i] < 0))
            return STMG_EINVAL;
        maxm = std::max(maxm, m_of[i]);
    }
    std::stable_sort(ord.begin(), ord.end(), [&](int x, int y) { return m_of[x] > m_of[y]; });
    // launch parameters of the persistent factorization: LDS budget from the
    // workgroups per CU, panel width per matrix from its size class (halved
    // until the panel fits the budget)
    constexpr size_t CU_LDS_BYTES = 160 * 1024;
    const bool f64 = prec == STMG_F64;
    LuTune tune = LU_TUNED[tune_index(prec)];
    if (cfg) tune = *cfg;
    const bool per_class = tune.wg_per_cu == 0;
    size_t budget = per_class ? 0 : CU_LDS_BYTES / (size_t)std::max(1, tune.wg_per_cu) - 1024;
    std::vector<int> nbv(batch, 4);
    if (!solve && !per_class) {
        // the largest matrix must fit with the narrowest panel, within the
        // dynamic LDS a workgroup may take
        int dev = 0, lds = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds = 65536;
        const size_t max_lds = lds > 8192 ? (size_t)lds - 8192 : (size_t)lds;
        budget = std::min(std::max(budget, lu_panel_lds_bytes(4, maxm, f64)), std::max(max_lds, (size_t)0));
        if (lu_panel_lds_bytes(4, maxm, f64) > budget) return STMG_EINVAL;
        for (int i = 0; i < batch; ++i) {
            const int m = m_of[ord[i]];
            int nb = tune.nb[size_class(m)];
            while (nb > 4 && lu_panel_lds_bytes(nb, m, f64) > budget) nb /= 2;
            nbv[i] = nb;
        }
    }
    // host image of the device metadata: [header: queue counter | m, nb (one
    // 8-byte slot per matrix) | a_off | p_off | b_off]
    const size_t hdr_words = META_HEADER_BYTES / sizeof(long long);
    std::vector<long long> meta(hdr_words + (size_t)4 * batch, 0);
    int *ms = reinterpret_cast<int *>(meta.data() + hdr_words);
    int *nbs = ms + batch;
    long long *ao = meta.data() + hdr_words + batch, *po = ao + batch, *bo = po + batch;
    for (int i = 0; i < batch; ++i) {
        ms[i] = m_of[ord[i]];
        nbs[i] = nbv[i];
        ao[i] = a_off[ord[i]];
        po[i] = p_off[ord[i]];
        bo[i] = solve ? b_off[ord[i]] : 0;
    }
    hipStream_t s = (hipStream_t)stream;
    DevAlloc own;
    unsigned char *dmeta = nullptr;
    if (staging == MetaStaging::Fixed) {
        void *p = nullptr;
        const int rc = scratch_address(&p);
        if (rc != STMG_OK) return rc;
        dmeta = static_cast<unsigned char *>(p);
    } else {
        if (hipMalloc(&own.p, batched_lu_meta_bytes(batch)) != hipSuccess) {
            own.p = nullptr;
            (void)hipGetLastError();
            return STMG_ENOMEM;
        }
        dmeta = static_cast<unsigned char *>(own.p);
    }
    // the copy also clears the queue counter in the header
    int *dcounter = reinterpret_cast<int *>(dmeta);
    const int *dm = reinterpret_cast<const int *>(dmeta + META_HEADER_BYTES);
    const int *dnb = dm + batch;
    const long long *da = reinterpret_cast<const long long *>(dmeta + META_HEADER_BYTES) + batch, *dp = da + batch,
                    *db = dp + batch;
    if (hipMemcpyAsync(dmeta, meta.data(), batched_lu_meta_bytes(batch), hipMemcpyHostToDevice, s) != hipSuccess) {
        (void)hipStreamSynchronize(s);
        return STMG_EHIP;
    }
    LuBatch vb{maxm, dm, da, dp};
    hipError_t e = hipSuccess;
    if (solve) {
        if (prec == STMG_F64)
            e = launch_batched_solve<double>((const double *)A, piv, maxm, batch, vb, db, (double *)b, s);
        else
            e = launch_batched_solve<float>((const float *)A, piv, maxm, batch, vb, db, (float *)b, s);
    } else if (!per_class) {
        // one persistent launch for the whole batch, largest matrices first
        LuQueue q{batch, dm, da, dp, dnb, dcounter};
        const int grid = std::min(batch, device_cus() * std::max(1, (int)(CU_LDS_BYTES / (budget + 1024))));
        if (prec == STMG_F64) e = launch_lu_queue<double>((double *)A, piv, q, budget, grid, tune.threads, info, s);
        else e = launch_lu_queue<float>((float *)A, piv, q, budget, grid, tune.threads, info, s, op);
    } else {
        int dev = 0, lds = 65536;
        if (hipGetDevice(&dev) != hipSuccess ||
            hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev) != hipSuccess)
            lds = 65536;
        const size_t max_lds = lds > 8192 ? (size_t)lds - 8192 : (size_t)lds;
        // one launch per size class (consecutive sorted matrices within a
        // factor 2 of the class's largest), each sizing its LDS panel for its
        // own largest matrix
        for (int c0 = 0; c0 < batch && e == hipSuccess;) {
            const int m0 = ms[c0];
            int c1 = c0 + 1;
            while (c1 < batch && 2 * ms[c1] > m0) ++c1;
            LuBatch vc{m0, dm + c0, da + c0, dp + c0};
            if (prec == STMG_F64) e = launch_lu<double>((double *)A, piv, m0, c1 - c0, info, max_lds, s, &vc);
            else e = launch_lu<float>((float *)A, piv, m0, c1 - c0, info, max_lds, s, &vc, op);
            c0 = c1;
        }
    }
    // the metadata must outlive the kernels (per-call allocation freed on
    // return; the fixed array is reused by the next call)
    const hipError_t es = hipStreamSynchronize(s);
    if (e == hipErrorInvalidConfiguration) return STMG_EINVAL;
    if (e != hipSuccess || es != hipSuccess) return STMG_EHIP;
    return STMG_OK;
}

} // namespace stmg
