// device.h - the device primitives the host engine issues, implemented in
// device.hip for gfx950.  Every call is asynchronous on the context stream
// unless it says otherwise; integer returns are 0 on success.
//
// Work is described by flat task lists (uploaded once per bond and reused by
// every Davidson product) that reference up to kMaxBufs base pointers; an
// offset is counted in elements of the buffer's element type.
#pragma once
#include <cstddef>
#include <cstdint>

namespace dmrgdev {

constexpr int kMaxBufs = 8;

struct Ctx;

int ctx_create(int device, void* stream, Ctx** out, char* err, size_t errlen);
void ctx_destroy(Ctx* c);
const char* last_error(Ctx* c);

void* alloc(Ctx* c, size_t bytes);          // nullptr on failure
void release(Ctx* c, void* p);
int h2d(Ctx* c, void* dst, const void* src, size_t bytes);   // returns when src may be reused
// Stream-ordered upload: src is copied into a pinned staging arena at once
// (src may be reused on return) and the device copy is queued on the stream.
// The arena is recycled at the next full stream synchronisation.
int h2d_async(Ctx* c, void* dst, const void* src, size_t bytes);
int d2h(Ctx* c, void* dst, const void* src, size_t bytes);   // synchronous
int d2d(Ctx* c, void* dst, const void* src, size_t bytes);
int fill(Ctx* c, double* x, int64_t n, double v);
int sync(Ctx* c);
// Make the context's device current on the calling host thread.
int bind(Ctx* c);

// Static device scratch (no allocation): the device address of this
// device's fixed array of kStaticScratchBytes, resolved when the context was
// created.  Shared by every context on the device; its contents persist
// between uses.
constexpr size_t kStaticScratchBytes = (size_t)64 << 20;
void* static_scratch(Ctx* c, size_t* bytes);

// timing on the context stream
int event_record(Ctx* c, int slot);                   // slot < 64
double event_elapsed(Ctx* c, int slot0, int slot1);   // seconds, synchronises

// ---------------------------------------------------------------- GEMM
// One output tile per task:
//   C[m0:m0+mt, n0:n0+nt] = beta*C + sum_chunks alpha * op(A)[m0.., :K] op(B)[:K, n0..]
// op(A) is M x K: stored row-major M x K (a_trans = 0) or K x M (a_trans = 1).
// op(B) is K x N: stored row-major K x N (b_trans = 0) or N x K (b_trans = 1).
// Offsets point at the block origins (row 0, column 0 of op(.)).
struct GemmChunk {
    double alpha;
    int64_t a_off, b_off;
    int32_t lda, ldb, K;
    uint8_t a_buf, b_buf, a_trans, b_trans;
};
// c_local = 1: C is a compact 64 x 64 partial tile at c_off (row stride
// kTileN, indexed from the tile origin) instead of the output block.
struct GemmTask {
    int64_t c_off;
    int32_t ldc, m0, n0, mt, nt;
    int32_t chunk_begin, chunk_end;
    uint8_t c_buf, beta, c_local, pad1;
};
// Split-K reduction: dst tile (mt x nt at dst_off, row stride ld) =
// (beta ? dst : 0) + sum of nslots consecutive partial tiles from slot0,
// summed in slot order (deterministic).
struct RedTask {
    int64_t dst_off;
    int32_t ld, mt, nt, slot0, nslots;
    uint8_t dst_buf, beta, pad0, pad1;
};
constexpr int kPartialBuf = 7;   // buffer index of the partial tiles
constexpr int kTileM = 64;
constexpr int kTileN = 64;

enum Prec { P_F64 = 0, P_F32 = 1, P_BF16 = 2 };

// Schedule of a persistent launch of `nwg` work-groups: work-group w runs
// tasks [wg_off[w], wg_off[w+1]) in order (wg_off is a device array of nwg + 1
// entries; work-group w lives on XCD w % 8); tasks [nfull, ntasks) have no
// chunks and only clear their tile.  A and B of one launch share a precision
// (ab_prec); C is c_prec.  Supported: (F64, F64), (F32, F32), (BF16, F32),
// (BF16, BF16).  Accumulation is FP64 for F64 operands and FP32 otherwise.
struct Sched {
    const int32_t* wg_off;
    int32_t nwg, nfull, ntasks;
};
// kind: which H_eff phase a launch is (only the kernel's name differs, for profiles)
enum GemmKind { GK_OTHER = 0, GK_HEFF_Z = 1, GK_HEFF_Y = 2 };
// ev_start / ev_stop (event slots, or -1): recorded by the kernel's own
// dispatch at its start and end, so that their interval is the kernel alone.
int gemm(Ctx* c, int ab_prec, int c_prec, void* const* bufs, const GemmTask* d_tasks, const Sched& sched,
         const GemmChunk* d_chunks, int kind = GK_OTHER, int ev_start = -1, int ev_stop = -1);
int gemm_reduce(Ctx* c, int c_prec, void* const* bufs, const RedTask* d_tasks, int ntasks);

// Grouped launch of several plans (independent solves advanced together):
// one descriptor per plan with its buffer table, task and chunk lists and
// schedule; work-group g runs plan p for prefix[p] <= g < prefix[p + 1] as
// that plan's work-group g - prefix[p].  d_plans and d_prefix (nplans + 1
// entries, prefix[nplans] = total_wg) are device arrays.
struct PlanDesc {
    void* bufs[kMaxBufs];
    const GemmTask* tasks;
    const GemmChunk* chunks;
    Sched sc;
};
int gemm_multi(Ctx* c, int ab_prec, int c_prec, const PlanDesc* d_plans, const int32_t* d_prefix, int nplans,
               int total_wg, int kind);
// split-K reductions of several plans: reduction x of plan p is block
// prefix[p] + x (prefix[nplans] = total)
struct RedDesc {
    void* bufs[kMaxBufs];
    const RedTask* reds;
};
int gemm_reduce_multi(Ctx* c, int c_prec, const RedDesc* d_plans, const int32_t* d_prefix, int nplans, int total);

// Cross-stream ordering (opaque event handles, no timing)
void* xevent_create(Ctx* c);             // nullptr on failure
void xevent_destroy(void* e);
int xevent_record(Ctx* c, void* e);      // record on c's stream
int xevent_wait(Ctx* c, void* e);        // c's stream waits for the last record of e
int xevent_sync(Ctx* c, void* e);        // the host waits for the last record of e
int ctx_device(Ctx* c);

// HIP graphs: capture the work queued on the context stream between begin and
// end (nothing runs meanwhile) into an executable graph; launch it on the
// stream as often as needed; destroy it when its buffers change.
int graph_begin(Ctx* c);
int graph_end(Ctx* c, void** exec);
int graph_launch(Ctx* c, void* exec);
void graph_destroy(void* exec);

// ------------------------------------------------------- linear combination
// dst[r0+r, c0+c] = sum_terms coef * src(r0+r, c0+c) with src(r, c) =
// S[r*ld + c], S[c*ld + r] (trans) or delta_rc (ident).  FP64.
struct LcTerm {
    double coef;
    int64_t src_off;
    int32_t ld;
    uint8_t buf, trans, ident, pad;
};
struct LcTask {
    int64_t dst_off;
    int32_t ld, r0, c0, mt, nt;
    int32_t t_begin, t_end;
    uint8_t buf, pad0, pad1, pad2;
};
constexpr int kLcTile = 32;
int lincomb(Ctx* c, double* const* bufs, const LcTask* d_tasks, int ntasks, const LcTerm* d_terms);

// -------------------------------------------------------- H_eff diagonal
// d[r0+r, c0+c] = sum_terms coef * a(r0+r) * b(c0+c), a(x) = A[a_off + x*a_step]
// (or 1 if a_ident), likewise b.  FP64.
struct DiagTerm {
    double coef;
    int64_t a_off, b_off;
    int32_t a_step, b_step;
    uint8_t a_buf, b_buf, a_ident, b_ident;
};
struct DiagTask {
    int64_t d_off;
    int32_t ld, r0, c0, mt, nt;
    int32_t t_begin, t_end;
};
int diag(Ctx* c, double* const* bufs, const DiagTask* d_tasks, int ntasks, const DiagTerm* d_terms);

// -------------------------------------------------- segment dot products
// partial[t] = coef_t * sum_{r < rows, c < cols} A[a_off + r*lda + c] * B[b_off + r*ldb + c]
// with A = bufs[a_buf], B = bufs[b_buf]; then out[o] = sum of partial[t] over
// t in [obeg[o], obeg[o+1]) in that order.  FP64, deterministic.
struct SegDot {
    double coef;
    int64_t a_off, b_off;
    int32_t rows, cols, lda, ldb;
    uint8_t a_buf, b_buf, pad0, pad1;
};
int seg_dots(Ctx* c, double* const* bufs, const SegDot* d_segs, int nseg, const int32_t* d_obeg, int nout,
             double* d_partial, double* d_out);

// ----------------------------------------------------- FP64 vector kernels
// V holds nvec vectors of length n at stride ldv.
// d_out[v * ostride] = V_v . w
int dots(Ctx* c, const double* V, int64_t ldv, int nvec, const double* w, int64_t n, double* d_out,
         int ostride = 1);
// out = (accumulate ? out : 0) + scale * sum_v coef[v] V_v      (coef on device)
int combine(Ctx* c, const double* V, int64_t ldv, int nvec, const double* d_coef, double scale,
            int64_t n, double* out, int accumulate);
// r = hx - theta * x ; also writes |r|^2 to d_norm2
int residual(Ctx* c, const double* hx, const double* x, const double* d_theta, int64_t n,
             double* r, double* d_norm2);
// t = r / (d - theta), |d - theta| clamped to >= 1e-12 keeping its sign
int precond(Ctx* c, const double* r, const double* d, const double* d_theta, int64_t n, double* t);
// x *= 1/sqrt(*d_norm2)
int scale_inv_norm(Ctx* c, double* x, int64_t n, const double* d_norm2);
// y = x * (1/sqrt(*d_norm2))
int copy_scaled_inv_norm(Ctx* c, const double* x, int64_t n, const double* d_norm2, double* y);
// lowest eigenpair of the symmetric k x k matrix whose lower triangle
// (G[i][j], j <= i) is given at row stride ldg
int small_eigh(Ctx* c, const double* d_G, int k, int ldg, double* d_theta, double* d_s);
// type conversion of n elements
int convert(Ctx* c, int from_prec, const void* src, int to_prec, void* dst, int64_t n);

// ------------------------------------------------- dense symmetric eigen
// A (n x n, symmetric) is overwritten with eigenvectors: row e of the
// row-major array is the eigenvector of w[e]; w ascending.
int syevd(Ctx* c, int n, double* A, double* w);
// `count` symmetric P x P matrices at stride P*P, solved together (same
// output convention; w at stride P).
int syevd_batched(Ctx* c, int P, int count, double* A, double* w);
// Buckets j = 0..nb-1 of count[j] padded P[j] x P[j] matrices at A + aoff[j]
// (eigenvalues at w + woff[j]), solved concurrently; ordered after all prior
// work of the context stream, and later work waits for them.
int syevd_buckets(Ctx* c, int nb, const int* P, const int* count, double* A, const int64_t* aoff, double* w,
                  const int64_t* woff);
// Prepare padded slots: for slot s (base + s*P*P, real size n[s]) write 0
// outside the leading n x n block and -1 on the padding diagonal, so the
// padding eigenpairs are (-1, unit vectors of the padding rows).
int pad_init(Ctx* c, double* base, int P, int count, const int32_t* d_n);
// U[r, col] = s_col * E[idx[col] * stride + r] for r < n (E rows = eigenvectors),
// s_col = +-1 making the first largest-magnitude entry (r < n) positive.
int gather_evecs(Ctx* c, const double* E, int n, int stride, const int32_t* d_idx, int k, double* U);

}  // namespace dmrgdev
