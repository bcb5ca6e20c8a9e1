// Launch wrappers of the basis-recursion, evaluation and Lanczos kernels.
#pragma once

#include "ops.hpp"

namespace ihs {

struct EvalItem {  // one lambda of an evaluation request
  int32_t l;       // interval
  int32_t k;       // basis terms of that interval
  double tau;      // step size
  double mu;       // tau * (lam - ref)
};

// per: column blocks per C block (0: every block takes the one C).
void launch_seed_rhs(const double* C, int64_t d, int64_t K, int na, double* R, int64_t ldr,
                     hipStream_t st, int per = 0);
void launch_store_first(const double* U, int64_t ldu, int64_t d, int64_t K, int na,
                        const int32_t* ids, int64_t kcap, double* basis, hipStream_t st);
void launch_form_r(const double* W, const double* U, int64_t ld, int64_t d, int64_t K, int na,
                   int i, const double* tau, const double* ref, double* R, hipStream_t st);
int launch_update(const double* U, const double* Z, double* Unew, int64_t ld, int64_t d, int64_t K,
                  int na, int i, const int32_t* ids, int64_t kcap, double* basis,
                  const double* mu_lo, const double* mu_hi, double* partial, hipStream_t st);
void launch_compact(const double* Src, double* Dst, int64_t ld, int64_t d, int64_t cw, int na_new,
                    const int32_t* keep, hipStream_t st);
void launch_eval(const double* basis, int64_t kcap, int64_t d, int64_t K, const EvalItem* items,
                 int64_t T, void* X, int64_t ldx, int x_dtype, hipStream_t st);
void launch_lanczos_start(uint64_t seed, int64_t d, int na, int64_t ld, double* Q0, hipStream_t st);
void launch_add_shift(double* S, const double* T, int64_t d, int na, int64_t ld, const double* lam0,
                      hipStream_t st);
void launch_lanczos_orth(double* Q, double* Wv, int64_t d, int na, int64_t ld, int j, int J,
                         double* alpha, double* beta, hipStream_t st);

// y_b = L_{map[b]} x_b (transpose = false) or L_{map[b]}^T x_b (true) for nb
// lower-triangular d x d factors; x_b, y_b are columns b of X, Y.  nv = 2:
// columns b and b + nb/2 use the same factor map[b] (map holds nb/2 entries)
// and each factor is read once for both.
// scratch: trmv_scratch_doubles(d, nb) doubles (used when transpose is set).
void launch_trmv(const double* L, int64_t d, const int32_t* map, int nb, bool transpose,
                 const double* X, int64_t ldx, double* Y, int64_t ldy, double* scratch,
                 hipStream_t st, int nv = 1);
// The same on the n x n diagonal block of each factor that starts at L (row
// stride ldl, factor b at L + map[b] * ms): X and Y hold the block's rows.
void launch_trmv_block(const double* L, int64_t n, int64_t ldl, int64_t ms, const int32_t* map,
                       int nb, bool transpose, const double* X, int64_t ldx, double* Y,
                       int64_t ldy, double* scratch, hipStream_t st, int nv = 1);
int64_t trmv_scratch_doubles(int64_t d, int nb);

}  // namespace ihs
