// Grid transfers between two levels of the hp hierarchy (internal).
#pragma once

#include "context.h"
#include "vec_ops.h"

namespace stmg {

struct HostCsr {
    int nrows = 0, ncols = 0;
    std::vector<int> rowptr, col;
    std::vector<double> val;
    long long counted_nnz = -1;   // >= 0: only the sizes were computed (arrays empty)
    long long nnz() const { return counted_nnz >= 0 ? counted_nnz : (long long)col.size(); }
};

struct DevCsr {
    int nrows = 0, ncols = 0;
    long long nnz = 0;
    DevBuf rowptr, col, val64, val32;
    void upload(const HostCsr &A);
};

// count_only: rows, columns and the number of entries, no arrays (used when a
// context is only measured)
HostCsr transpose(const HostCsr &A);
HostCsr velocity_prolongation(const Level &f, const Level &c, char kind, bool count_only = false);
HostCsr state_interpolation(const Level &f, const Level &c, char kind, bool count_only = false);
HostCsr pressure_prolongation(const Level &f, const Level &c, char kind, bool count_only = false);

struct Transfer {
    char kind = 'h';
    DevCsr vel, velT, pres, presT, state;
    DevBuf Pt64, Pt32, PtT64, PtT32, It64, It32;
    void build(const Level &f, const Level &c, char kind);
    // yf = P xc + beta yf  (slab vectors)
    template <typename T> void prolongate(const Level &f, const Level &c, const T *xc, T *yf, T beta, hipStream_t s) const;
    // yc = P^T xf
    template <typename T> void restrict_(const Level &f, const Level &c, const T *xf, T *yc, hipStream_t s) const;
    // coarse velocity state (all time nodes) from the fine one
    template <typename T>
    void interpolate_state(const Level &f, const Level &c, const T *vf, T *vc, hipStream_t s) const;
};

} // namespace stmg
