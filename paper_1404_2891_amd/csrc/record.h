// Recording of the device work of one pencil, so that the work of many pencils can be launched
// together.  While a log is installed on the calling thread (op_log()), the product, element-wise
// and copy helpers append what they would enqueue instead of enqueueing it; a batch of pencils
// records one phase of its iteration for every member and then launches the logs side by side:
// operations at the same position of the members' logs that run the same kernel with compatible
// parameters become one grouped launch (each member's operands read from a device table), the rest
// run one by one.  Every member's operations keep their order, and members are independent, so any
// such merge is exact.
#pragma once

#include <functional>
#include <vector>

#include "common.h"
#include "gemm.h"

namespace fm {

enum RecKind { REC_NOP = 0, REC_GEMM = 1, REC_EW = 2, REC_COPY = 3, REC_MARK = 4, REC_OTHER = 5 };

// Element-wise kernels that have a grouped form (solve.hip).
enum EwKind { EW_GATHER_F32 = 0, EW_GATHER_F64, EW_ACCUM_F32, EW_ACCUM_F64, EW_RESIDUAL, EW_COPY_CM, EW_RITZ, EW_CHOL,
              EW_WORDS, EW_CHOL_BIG, EW_COUNT };

// EW_WORDS: a copy of `words` 4-byte words between device buffers (both 4-byte aligned); with a
// grouped launch, the small transfers of many pencils go through one staging buffer and one
// host <-> device copy.
struct WordsArgs {
    const unsigned* src;
    unsigned* dst;
    long words;
};

constexpr int EW_ARG_BYTES = 192;

struct RecOp {
    int kind = REC_NOP;
    // REC_GEMM: the product (never grouped itself) and its element type
    GemmOp g;
    bool dbl = false;
    // REC_EW: the kernel, its argument block, and the member's grid (blocks along x, extent along y)
    int ew = 0;
    alignas(16) unsigned char args[EW_ARG_BYTES];
    unsigned bx = 0, by = 1;
    // REC_COPY: an asynchronous copy
    void* dst = nullptr;
    const void* src = nullptr;
    size_t bytes = 0;
    hipMemcpyKind dir = hipMemcpyDefault;
    // REC_MARK: start or stop of a timed phase (the algorithmic flops at the stop)
    int phase = 0;
    bool start = false;
    double flops = 0.0;
    // REC_OTHER: the launch itself, on a given stream
    std::function<int(hipStream_t)> run;
};

struct OpLog {
    std::vector<RecOp> ops;
    // the block sweeps of the multi-RHS solves take this many steps, empty ones beyond a pencil's
    // own count, so that the steps of pencils of different orders line up
    int pad_steps = 0;
    void nop() { ops.emplace_back(); }
    void other(std::function<int(hipStream_t)> f) {
        RecOp r;
        r.kind = REC_OTHER;
        r.run = std::move(f);
        ops.push_back(std::move(r));
    }
};

// The calling thread's log (nullptr: enqueue directly).
inline OpLog*& op_log() {
    static thread_local OpLog* log = nullptr;
    return log;
}

// Asynchronous copy on st, or recorded.
inline int copy_async(void* dst, const void* src, size_t bytes, hipMemcpyKind dir, hipStream_t st) {
    if (OpLog* L = op_log()) {
        RecOp r;
        r.kind = REC_COPY;
        r.dst = dst;
        r.src = src;
        r.bytes = bytes;
        r.dir = dir;
        L->ops.push_back(std::move(r));
        return 0;
    }
    FM_HIP(hipMemcpyAsync(dst, src, bytes, dir, st));
    return 0;
}

// Grouped product: one launch for members (their GemmGroup entries in `groups` on the device) that
// share proto's layout, conjugation, alpha and beta; max_* size the grid (gemm.hip).
template <typename T>
int gemm_grouped(const GemmOp& proto, const GemmGroup* groups, int ngroups, int max_M, int max_N, int max_K,
                 int max_batch, int max_splitk, hipStream_t st);

// The grouped-product entry of one product (with its split-K partition) (gemm.hip).
template <typename T>
GemmGroup gemm_member(const GemmOp& op);

// Grouped launch of element-wise kernel `ew` over ngroups argument blocks (device table of
// ngroups blocks of the kernel's argument size) (solve.hip).
int ew_grouped(int ew, const void* table, int ngroups, unsigned max_bx, unsigned max_by, hipStream_t st);
size_t ew_arg_size(int ew);

}  // namespace fm
