// Internal declarations shared by the runtime translation units.
#pragma once

#include <hip/hip_runtime.h>

#include <mutex>
#include <vector>

#include "blip.h"
#include "blip_launch.hpp"

namespace blip {

constexpr uint32_t kTableMagic = 0xB11F7AB1u;

enum ElemKind { ELEM_F32 = 0, ELEM_BF16 = 1, ELEM_F16 = 2 };

// A tuned launch shape for npos in [lo, hi].
struct TuneEntry {
    int64_t lo, hi;
    int P, OE;
};

// Acceptance-ratio epilogue arguments (blip_eval_ratio*).
struct RatioArgs {
    const double* inv_rows;
    int64_t inv_ld;
    const int64_t* row_of;
    double* ratio;
    double* gratio;
    double* lratio;
};

// Launch-shape tables kept per table: single blocks and sorted batches, each
// with and without the acceptance-ratio epilogue (a ratio mode falls back to
// its plain mode's shapes when it has none of its own).
enum TuneMode { MODE_BLOCK = 0, MODE_BATCHED = 1, MODE_BLOCK_RATIO = 2, MODE_BATCHED_RATIO = 3,
                MODE_COUNT = 4 };

}  // namespace blip

struct blip_table_s {
    uint32_t magic;
    int device;
    int ncu;             // compute units of the device
    double A[9];         // lattice rows a_1, a_2, a_3
    double G[9];         // A^{-1}
    double M[9];         // M_cd = n_d G_cd
    double g6[6];        // g_11, g_22, g_33, g_12, g_13, g_23
    double k[3];         // k-point (complex tables with a Bloch factor)
    int n[3];
    int L;               // orbitals
    int W;               // table elements per site: L (real) or 2L (complex)
    blip_dtype storage;
    int elem;            // blip::ElemKind
    int esize;           // bytes per table element
    bool complex_;
    bool bloch;
    bool ortho;          // lattice rows along the axes: metric is diagonal
    int64_t row_bytes;   // W * esize rounded up to 128 bytes
    int64_t nrows;       // n1 * n2 * n3
    size_t table_bytes;
    char* d_table;
    float out_scale;     // 2^-e for FP16 tables stored as a * 2^e
    // spatial bins for batch sorting: bricks of 2^bshift cells per side,
    // numbered by their rank along a Morton (Z-order) curve
    int bshift;
    int nb[3];
    int nbins;
    int* d_brick_rank;   // [nb0][nb1][nb2] -> Morton rank
    mutable std::mutex tune_mu;
    std::vector<blip::TuneEntry> tune[blip::MODE_COUNT];   // indexed by blip::TuneMode
};

namespace blip {

int fail(int code, const char* fmt, ...) __attribute__((format(printf, 2, 3)));
int fail_hip(hipError_t e, const char* what);
bool aligned16(const void* p);
bool table_ok(const blip_table_s* t);
void fill_table_args(const blip_table_s* t, KArgs& a);
hipError_t dispatch(const blip_table_s* t, const KArgs& a, const Cfg& c, hipStream_t s);
void choose_shape(const blip_table_s* t, int mode, int64_t npos, int& P, int& OE);
void set_tuned(blip_table_s* t, int mode, int64_t npos, int P, int OE);
// Launch the tiled (or FP64-accumulate) kernel.  perm/dev_count select the
// sorted persistent form used for batches; grid is then the workgroup count.
int launch_tiled(const blip_table_s* t, const double* pos, int64_t npos, void* val, void* grad,
                 void* lap, int kind, int P, int OE, const int* perm, const double* spos,
                 const int64_t* dev_count, int* xcd_next, int grid, bool chunk_major,
                 hipStream_t s, const RatioArgs* ratio = nullptr);
bool valid_oe(const blip_table_s* t, int OE);
int check_eval_args(blip_table t, const double* pos, int64_t npos, void* val, void* grad,
                    void* lap);
// Kernel kind and shape overrides from blip_eval_ex options (NULL: tuned tiled).
int eval_opts(blip_table t, const blip_eval_opts* opts, int& kind, int& P, int& OE);
// blip_eval_ex without the C-ABI wrapper.
int eval_common(blip_table t, const double* pos, int64_t npos, void* val, void* grad,
                void* lap, const blip_eval_opts* opts, void* stream);
int check_ratio_args(blip_table t, int64_t npos, const double* pos, const double* inv_rows,
                     int64_t inv_ld, const int64_t* row_of, double* ratio, double* grad_ratio,
                     double* lap_ratio);
// P and o for the ratio epilogue (P <= 16, at most 16 orbital chunks).
int ratio_shape(const blip_table_s* t, int mode, int64_t npos, int& P, int& OE);
void make_cfg(const blip_table_s* t, int kind, int P, int OE, bool full, int64_t grid, Cfg& c,
              KArgs& a);
int upload_table(blip_table_s* t, const void* host);
int make_brick_ranks(blip_table_s* t);

}  // namespace blip
