// Kernel launchers (host side) used by the plan executor.
#pragma once

#include <hip/hip_runtime.h>

#include <vector>

#include "../../include/qgt_block.h"
#include "qgt_internal.h"

namespace qgt {

// Record an error for qgt_last_error() and return s; check the last launch.
qgt_status report_error(qgt_status s, const char* msg);
qgt_status report_launch(const char* what);

void launch_bind(const BindArgs& a, int nprob, ProbPtrs* dst, hipStream_t s);
void launch_fill_i32(int32_t* p, int n, int32_t v, hipStream_t s);
void launch_eloc(const ProbDev* probs, const ProbPtrs* ptrs, char* ws, int nprob, hipStream_t s);
void launch_colpass(int dt, int phase, const ColTile* tiles, int ntiles, int RC, const BlockDev* blocks,
                    const ProbDev* probs, const ProbPtrs* ptrs, char* ws, double2* part, hipStream_t s);
void launch_block_trace(const BlockDev* blocks, const ProbDev* probs, char* ws, double* trace, int nblocks,
                        hipStream_t s);
void launch_mudot(const int32_t* glist, int n, const BlockDev* blocks, const ProbDev* probs, char* ws,
                  double2* bscal, hipStream_t s);
void launch_rowpass(int dt, int phase, const RowItem* items, int nitems, const BlockDev* blocks,
                    const ProbDev* probs, const ProbPtrs* ptrs, char* ws, const double2* bscal, hipStream_t s);
void launch_pack(int dt, int prec, const int32_t* glist, int n, int64_t max_mtiles, int ygrid, const BlockDev* blocks,
                 const ProbDev* probs, const ProbPtrs* ptrs, char* ws, int form, hipStream_t s);
void launch_cg(int phase, const BlockDev* blocks, char* ws, CgScal* cg, double rtol, int iters, int32_t* status,
               int nblocks, hipStream_t s);
void launch_init_solve(const BlockDev* blocks, const ProbDev* probs, char* ws, int nblocks, int64_t max_mpad,
                       hipStream_t s);
void launch_scatter_p(const BlockDev* blocks, const ProbPtrs* ptrs, char* ws, int nblocks, int64_t max_nb,
                      hipStream_t s);
void launch_gram_duo(const GramItem* items, int maxlen, const int32_t* xcd_start, const int32_t* xcd_len,
                     const BlockDev* blocks, char* ws, hipStream_t s);
void launch_gram_wide(const GramItem* items, int maxlen, const int32_t* xcd_start, const int32_t* xcd_len,
                      const BlockDev* blocks, char* ws, hipStream_t s);
void launch_gram(int prec, const GramItem* items, int maxlen, const int32_t* xcd_start, const int32_t* xcd_len,
                 const BlockDev* blocks, char* ws, double2* part, hipStream_t s);
void launch_gram_splitk_reduce(const SplitItem* items, int n, const BlockDev* blocks, char* ws, const double2* part,
                               hipStream_t s);
void launch_potrf(const int32_t* glist, int n, const BlockDev* blocks, char* ws, int k, int32_t* status,
                  int32_t* floors, hipStream_t s);
void launch_tile_gemm(int mode, const int4* tasks, int n, const BlockDev* blocks, char* ws, int k, hipStream_t s);
void launch_chol(const CholTask* tasks, const int32_t* qoff, int nq, int ntasks, int nwg, const BlockDev* blocks,
                 char* ws, int* state, int* ctl, int32_t* status, int32_t* floors, hipStream_t s);
void launch_trsv_reset(const BlockDev* blocks, char* ws, int nblocks, int64_t max_mpad, hipStream_t s);
void launch_trsv(int dir, const int2* tmap, int ntickets, const BlockDev* blocks, char* ws, int* counter,
                 int32_t* status, hipStream_t s);

void launch_block_inverse_sums(const BlockDev* blocks, const std::vector<int>& glist, const std::vector<int64_t>& m,
                               const char* ws, double2* X, int64_t ldx, const double2* Bref, int64_t ldb, int64_t n_p,
                               double* part, double* part2, double* out, hipStream_t s);

void launch_dense(int mode, const DenseArgs& a, hipStream_t s);  // mode 0 FWD, 1 BWD
void launch_jac_rows(int dt, const JacArgs& a, hipStream_t s);
void launch_conv(int mode, const ConvArgs& a, hipStream_t s);  // mode 0 FWD, 1 BWD
void launch_conv_dk(int dt, const ConvDkArgs& a, int n_layers, hipStream_t s);

}  // namespace qgt
