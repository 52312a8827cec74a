// Launchers of the HIP kernels (defined in kernels.hip).
#pragma once
#include <hip/hip_runtime.h>

#include "desc.hpp"

namespace h2 {

enum GemmKind { GEMM_NN = 0, GEMM_NT = 1, GEMM_TN = 2, GEMM_TT = 3 };

// GEMM tuning table: capacity buckets (largest block dimension <= 256, 512,
// 1024, 2048, larger), and per (layout, FP32, bucket) the workgroups per shift,
// the tile-order group and the tile size (64 or 128).
constexpr int GEMM_BUCKETS = 5;
int gemm_bucket(int cap);
void set_gemm_tuning(int layout, int f32, int bucket, int grid, int group_m, int tile);
void get_gemm_tuning(int layout, int f32, int bucket, int* grid, int* group_m, int* tile);

void launch_fill(double* p, int64_t n, double v, hipStream_t st);
void launch_fill_int(int* p, int64_t n, int v, hipStream_t st);
// prefix: device scratch of at least nshift * (nitems + 1) ints (the per-shift tile counts)
void launch_gemm(int kind, const GItem* items, int nitems, const GTerm* terms, const BufTab& bt, const SizeTab& sz,
                 int mcap, int ncap, int nshift, int* prefix, hipStream_t st);
void launch_copyback(const CopyItem* items, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st);
void launch_copyback_t(const CopyItem* items, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st);
void launch_matsum(const SumItem* items, int nitems, const int* src, const BufTab& bt, const SizeTab& sz, int cap,
                   int nshift, hipStream_t st);
void launch_pchol_init(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st);
// tau2c: squared truncation budget of every cluster of the level
void launch_pchol_panel(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, const double* tau2c, int* more,
                        int cap, int nshift, hipStream_t st);
void launch_pchol_finish(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st);
void launch_hqr_panel(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int it, int* more, int nshift,
                      hipStream_t st);
void launch_eye(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st);
void launch_ldl_init(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int nshift, hipStream_t st);
void launch_ldl_panel(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz, int* status,
                      int* more, int nshift, hipStream_t st);
void launch_ldl_prep(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz,
                     unsigned long long* nu, int nshift, hipStream_t st);
void launch_diag_inv(const int* clusters, int n, const int* diag_blk, const BufTab& bt, const SizeTab& sz, int cap,
                     int nshift, hipStream_t st);
void launch_set_block(const int* clusters, int n, const SizeTab& sz, int ib, int use_t, int nshift, hipStream_t st);
void launch_ut_prep(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st);
void launch_ut_diag_inv(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift,
                        hipStream_t st);
void launch_kform(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int cap, int nshift, hipStream_t st);
void launch_zero_clusters(const int* clusters, int n, const BufTab& bt, int buf, int cap, int nshift, hipStream_t st);
int inv_block();
void launch_hqr_apply(const int* clusters, int n, const BufTab& bt, const SizeTab& sz, int tmax, int nshift, hipStream_t st);
int hqr_max_rows();              // largest cluster dimension the LDS-resident Householder panel takes
int ldl_panel_min(int cap);      // fewest pivots an LDL panel takes unless it reaches R
void launch_colour_max(const int* clusters, int n, const SizeTab& sz, int* out, int nshift, hipStream_t st);
constexpr int PCHOL_NB = 32;     // pivots per pivoted-Cholesky panel
constexpr int HQR_NB = 8;        // widest Householder panel (columns held in LDS)
void launch_merge_sizes(const SizeTab& sz, int Np, int nshift, hipStream_t st);
void launch_gather(const GatherItem* items, int n, const BufTab& bt, const SizeTab& sz, int pcap, int nshift, hipStream_t st);
void launch_merge_nn(const GatherItem* items, int n, const BufTab& bt, const SizeTab& sz, int pcap, int nshift,
                     hipStream_t st);
void launch_next_sizes(const SizeTab& sz, int nshift, hipStream_t st);
void launch_leaf_init(const BufTab& bt, int nblk, const int* blk_diag_m, const double* sigma, int cap, int nshift,
                      hipStream_t st);
void launch_sizes_init(const SizeTab& sz, const int* m0, int nshift, hipStream_t st);
void launch_row_abs_sum(const double* X, int64_t n, int dim, int kind, double p0, double p1, double* rad,
                        hipStream_t st);
void launch_kernel_blocks(double* out, int64_t bstride, int ld, const int* bi, const int* bj, int nblk,
                          const int64_t* start, const int* msz, const double* X, int dim, int kind, double diag,
                          double p0, double p1, int* bad, hipStream_t st);

}  // namespace h2
