// device.hip - gfx950 kernels and launchers behind device.h.
//
// Hot path: `gemm` is a grouped, multi-chunk GEMM.  One work-group (4 waves)
// owns one 64x64 output tile of one sector block and accumulates every chunk
// (term x input sub-block) that lands on it, so an output is written once,
// without atomics.  Operands are staged through LDS in K slices and
// multiplied on the matrix cores: v_mfma_f64_16x16x4f64 (FP64),
// v_mfma_f32_16x16x4f32 (FP32) and v_mfma_f32_16x16x32_bf16 (BF16 operands,
// FP32 accumulation).  FP64 and BF16 slices go through registers into LDS
// (transposes resolved while staging, gemm_body); FP32 slices are loaded
// straight into LDS and transposed operands are read down their columns
// (gemm_body_f32dma).  Each wave holds a 32x32 quarter of the tile as 2x2
// MFMA blocks.
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <rocblas/rocblas.h>
#include <rocsolver/rocsolver.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <cstddef>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "device.h"

namespace dmrgdev {

// Fixed device scratch for callers that cannot allocate (static_scratch):
// every GPU the library runs on holds its own copy until the process ends.
// Host code never uses the array's name as an address: its device address is
// looked up once per device (scratch_addr) and used from there on.
static __device__ __align__(256) unsigned char scratch[kStaticScratchBytes];

constexpr int kSide = 4;

struct Ctx {
    int device = 0;
    hipStream_t stream = nullptr;
    bool own_stream = false;
    rocblas_handle blas = nullptr;
    hipEvent_t ev[64] = {};
    std::string err;
    // scratch for reductions and the eigensolver
    double* red = nullptr;
    size_t red_cap = 0;
    double* syev_e = nullptr;
    size_t syev_cap = 0;
    int* info = nullptr;
    size_t info_cap = 0;
    // side streams for concurrent eigensolver buckets (default priority)
    bool side_ready = false;
    hipStream_t side[4] = {};
    rocblas_handle side_blas[4] = {};
    hipEvent_t side_ev[4] = {}, fork_ev = nullptr;
    double* side_e[4] = {};
    int* side_info[4] = {};
    size_t side_ecap[4] = {}, side_icap[4] = {};
    // pinned staging arena for stream-ordered uploads
    char* stage = nullptr;
    size_t stage_cap = 0, stage_off = 0;
    // device address of this device's static scratch array
    void* scratch = nullptr;
};

static int seterr(Ctx* c, const char* what, hipError_t e) {
    c->err = std::string(what) + ": " + hipGetErrorString(e);
    return 1;
}
#define HIPCHK(c, x)                                  \
    do {                                              \
        hipError_t _e = (x);                          \
        if (_e != hipSuccess) return seterr(c, #x, _e); \
    } while (0)
#define LAUNCHCHK(c)                                                   \
    do {                                                               \
        hipError_t _e = hipGetLastError();                             \
        if (_e != hipSuccess) return seterr(c, "kernel launch", _e);   \
    } while (0)

int ctx_create(int device, void* stream, Ctx** out, char* err, size_t errlen) {
    auto fail = [&](const char* m) {
        if (err && errlen) snprintf(err, errlen, "%s", m);
        return 1;
    };
    int n = 0;
    if (hipGetDeviceCount(&n) != hipSuccess || n == 0) return fail("no HIP device visible");
    if (device < 0 || device >= n) return fail("device ordinal out of range");
    if (hipSetDevice(device) != hipSuccess) return fail("hipSetDevice failed");
    Ctx* c = new Ctx();
    c->device = device;
    if (stream) {
        c->stream = (hipStream_t)stream;
    } else {
        if (hipStreamCreateWithFlags(&c->stream, hipStreamNonBlocking) != hipSuccess) {
            delete c;
            return fail("hipStreamCreate failed");
        }
        c->own_stream = true;
    }
    for (auto& e : c->ev)
        if (hipEventCreate(&e) != hipSuccess) {
            delete c;
            return fail("hipEventCreate failed");
        }
    if (rocblas_create_handle(&c->blas) != rocblas_status_success) {
        delete c;
        return fail("rocblas_create_handle failed");
    }
    rocblas_set_stream(c->blas, c->stream);
    if (hipMalloc(&c->info, sizeof(int)) != hipSuccess) {
        delete c;
        return fail("hipMalloc failed");
    }
    c->info_cap = 1;
    // device address of the static scratch on this device (with it current)
    {
        static std::mutex mu;
        static void* addr[256] = {};
        std::lock_guard<std::mutex> lock(mu);
        if (device >= 256) {
            ctx_destroy(c);
            return fail("device ordinal above 255");
        }
        if (!addr[device]) {
            void* p = nullptr;
            hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
            if (e != hipSuccess || !p) {
                ctx_destroy(c);
                return fail("hipGetSymbolAddress of the static scratch failed");
            }
            addr[device] = p;
        }
        c->scratch = addr[device];
    }
    *out = c;
    return 0;
}

void* static_scratch(Ctx* c, size_t* bytes) {
    if (bytes) *bytes = kStaticScratchBytes;
    return c->scratch;
}

void ctx_destroy(Ctx* c) {
    if (!c) return;
    hipSetDevice(c->device);
    hipStreamSynchronize(c->stream);
    if (c->blas) rocblas_destroy_handle(c->blas);
    for (auto& e : c->ev)
        if (e) hipEventDestroy(e);
    if (c->red) hipFree(c->red);
    if (c->syev_e) hipFree(c->syev_e);
    if (c->info) hipFree(c->info);
    if (c->stage) hipHostFree(c->stage);
    if (c->side_ready) {
        for (int i = 0; i < kSide; ++i) {
            hipStreamSynchronize(c->side[i]);
            rocblas_destroy_handle(c->side_blas[i]);
            hipEventDestroy(c->side_ev[i]);
            hipStreamDestroy(c->side[i]);
            if (c->side_e[i]) hipFree(c->side_e[i]);
            if (c->side_info[i]) hipFree(c->side_info[i]);
        }
        hipEventDestroy(c->fork_ev);
    }
    if (c->own_stream) hipStreamDestroy(c->stream);
    delete c;
}

const char* last_error(Ctx* c) { return c->err.c_str(); }

void* alloc(Ctx* c, size_t bytes) {
    void* p = nullptr;
    if (hipMalloc(&p, bytes ? bytes : 8) != hipSuccess) {
        hipGetLastError();
        c->err = "hipMalloc failed";
        return nullptr;
    }
    return p;
}
void release(Ctx*, void* p) {
    if (p) hipFree(p);
}
// every full synchronisation of the stream retires all queued staged copies
static int stream_sync(Ctx* c) {
    HIPCHK(c, hipStreamSynchronize(c->stream));
    c->stage_off = 0;
    return 0;
}
int h2d(Ctx* c, void* dst, const void* src, size_t bytes) {
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, c->stream));
    return stream_sync(c);
}
int h2d_async(Ctx* c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return 0;
    const size_t need = (bytes + 255) & ~(size_t)255;
    if (c->stage_off + need > c->stage_cap) {
        if (stream_sync(c)) return 1;
        if (need > c->stage_cap) {
            if (c->stage) HIPCHK(c, hipHostFree(c->stage));
            c->stage = nullptr;
            c->stage_cap = 0;
            const size_t cap = std::max<size_t>(need, (size_t)64 << 20);
            HIPCHK(c, hipHostMalloc((void**)&c->stage, cap, hipHostMallocDefault));
            c->stage_cap = cap;
        }
    }
    char* p = c->stage + c->stage_off;
    memcpy(p, src, bytes);
    c->stage_off += need;
    HIPCHK(c, hipMemcpyAsync(dst, p, bytes, hipMemcpyHostToDevice, c->stream));
    return 0;
}
int d2h(Ctx* c, void* dst, const void* src, size_t bytes) {
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToHost, c->stream));
    return stream_sync(c);
}
int d2d(Ctx* c, void* dst, const void* src, size_t bytes) {
    if (!bytes) return 0;
    HIPCHK(c, hipMemcpyAsync(dst, src, bytes, hipMemcpyDeviceToDevice, c->stream));
    return 0;
}
int sync(Ctx* c) { return stream_sync(c); }
int bind(Ctx* c) {
    HIPCHK(c, hipSetDevice(c->device));
    return 0;
}
void* xevent_create(Ctx* c) {
    hipEvent_t e = nullptr;
    if (hipEventCreateWithFlags(&e, hipEventDisableTiming) != hipSuccess) {
        c->err = "hipEventCreate failed";
        return nullptr;
    }
    return (void*)e;
}
void xevent_destroy(void* e) {
    if (e) hipEventDestroy((hipEvent_t)e);
}
int xevent_sync(Ctx* c, void* e) {
    HIPCHK(c, hipEventSynchronize((hipEvent_t)e));
    return 0;
}
int xevent_record(Ctx* c, void* e) {
    HIPCHK(c, hipEventRecord((hipEvent_t)e, c->stream));
    return 0;
}
int xevent_wait(Ctx* c, void* e) {
    HIPCHK(c, hipStreamWaitEvent(c->stream, (hipEvent_t)e, 0));
    return 0;
}
int ctx_device(Ctx* c) { return c->device; }

int graph_begin(Ctx* c) {
    HIPCHK(c, hipStreamBeginCapture(c->stream, hipStreamCaptureModeThreadLocal));
    return 0;
}
int graph_end(Ctx* c, void** exec) {
    *exec = nullptr;
    hipGraph_t g = nullptr;
    HIPCHK(c, hipStreamEndCapture(c->stream, &g));
    hipGraphExec_t x = nullptr;
    hipError_t e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
    hipGraphDestroy(g);
    if (e != hipSuccess) return seterr(c, "hipGraphInstantiate", e);
    *exec = (void*)x;
    return 0;
}
int graph_launch(Ctx* c, void* exec) {
    HIPCHK(c, hipGraphLaunch((hipGraphExec_t)exec, c->stream));
    return 0;
}
void graph_destroy(void* exec) {
    if (exec) hipGraphExecDestroy((hipGraphExec_t)exec);
}

int event_record(Ctx* c, int slot) {
    HIPCHK(c, hipEventRecord(c->ev[slot], c->stream));
    return 0;
}
double event_elapsed(Ctx* c, int a, int b) {
    float ms = 0.f;
    if (hipEventSynchronize(c->ev[b]) != hipSuccess) return 0.0;
    if (hipEventElapsedTime(&ms, c->ev[a], c->ev[b]) != hipSuccess) return 0.0;
    return ms * 1e-3;
}

// -------------------------------------------------------------- helpers
__global__ void k_fill(double* __restrict__ x, int64_t n, double v) {
    int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    int64_t s = (int64_t)gridDim.x * blockDim.x;
    for (; i < n; i += s) x[i] = v;
}
static unsigned grid_for(int64_t n, int per = 256, unsigned cap = 8192) {
    int64_t g = (n + per - 1) / per;
    if (g < 1) g = 1;
    if (g > cap) g = cap;
    return (unsigned)g;
}
int fill(Ctx* c, double* x, int64_t n, double v) {
    if (n <= 0) return 0;
    hipLaunchKernelGGL(k_fill, dim3(grid_for(n)), dim3(256), 0, c->stream, x, n, v);
    LAUNCHCHK(c);
    return 0;
}

// bf16 as raw 16-bit storage; round to nearest even on conversion
typedef unsigned short bf16_t;
__device__ __forceinline__ bf16_t f2bf(float f) {
    unsigned u = __float_as_uint(f);
    if ((u & 0x7f800000u) == 0x7f800000u) return (bf16_t)(u >> 16);   // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (bf16_t)(u >> 16);
}
__device__ __forceinline__ float bf2f(bf16_t h) { return __uint_as_float(((unsigned)h) << 16); }

// ================================================================ GEMM
struct Bufs {
    void* p[kMaxBufs];
};

typedef double d4_t __attribute__((ext_vector_type(4)));
typedef float f4_t __attribute__((ext_vector_type(4)));
typedef __bf16 bf8_t __attribute__((ext_vector_type(8)));

constexpr int TM = kTileM, TN = kTileN;   // 64 x 64 output tile
constexpr int NTH = 256;                  // 4 waves

// ---- FP64 / FP32: K slice 16, LDS As[k][m], Bs[k][n] (k-major, padded)
template <class T> struct MmaTraits;
// A operand: lane l holds A[l%16][l/16]; B operand: lane l holds B[l/16][l%16].
// Result register r of lane l is D[row(l, r)][l%16]; the row map differs
// between the FP64 and FP32 instructions (measured on gfx950).
// KS: K depth of one MFMA; a lane's operand fragment is 1 element (FP64, FP32)
// or 8 consecutive k (BF16: lane l holds k = 8 (l/16) .. +7).
template <> struct MmaTraits<double> {
    typedef d4_t acc_t;
    typedef double frag_t;
    typedef double scale_t;
    static constexpr int KS = 4;
    static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
        return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return (lane >> 4) + 4 * r; }
};
template <> struct MmaTraits<float> {
    typedef f4_t acc_t;
    typedef float frag_t;
    typedef float scale_t;
    static constexpr int KS = 4;
    static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
template <> struct MmaTraits<bf16_t> {
    typedef f4_t acc_t;
    typedef bf8_t frag_t;
    typedef float scale_t;
    static constexpr int KS = 32;
    static __device__ __forceinline__ acc_t mma(bf8_t a, bf8_t b, acc_t c) {
        return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
    }
    static __device__ __forceinline__ int row(int lane, int r) { return 4 * (lane >> 4) + r; }
};
// conversions of the output type (BF16 outputs round to nearest even)
template <class TC> __device__ __forceinline__ TC to_out(double v) { return (TC)v; }
template <> __device__ __forceinline__ bf16_t to_out<bf16_t>(double v) { return f2bf((float)v); }
template <class TC> __device__ __forceinline__ double from_out(TC v) { return (double)v; }
template <> __device__ __forceinline__ double from_out<bf16_t>(bf16_t v) { return (double)bf2f(v); }

// Register staging of one K slice for a 64-row operand tile (E = BK/4
// elements per thread).  LDS holds the tile as S[r][k] (k contiguous) with
// row stride LDK = BK + 4 floats (BK + 2 doubles): the MFMA fragment reads
// (16 rows x 4 consecutive k per wave) then hit distinct banks.  Global
// loads are coalesced along whichever dimension is contiguous in memory:
// "along K" (A plain, B transposed) or "along M/N" (A transposed, B plain).
// Operand loads go through raw buffer loads: a lane whose element lies
// outside the operand (ragged tile edge or past the chunk's K) gets an offset
// beyond the resource's range, and the hardware returns 0 for it without a
// memory access.  Offsets are 32-bit byte offsets from the operand block's
// own start (blocks are far below 2 GiB), so the per-element address work is
// a few 32-bit operations.
constexpr int kRecords = 0x7fffff00;   // resource range in bytes
constexpr int kOutside = 0x7fffff80;   // an offset past the range
__device__ __forceinline__ __amdgpu_buffer_rsrc_t make_rsrc(const void* base) {
    return __builtin_amdgcn_make_buffer_rsrc(const_cast<void*>(base), (short)0, kRecords, 0x00020000);
}
template <class T> __device__ __forceinline__ T bload(__amdgpu_buffer_rsrc_t r, int voff, int soff);
template <> __device__ __forceinline__ float bload<float>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(float, __builtin_amdgcn_raw_buffer_load_b32(r, voff, soff, 0));
}
template <> __device__ __forceinline__ double bload<double>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_bit_cast(double, __builtin_amdgcn_raw_buffer_load_b64(r, voff, soff, 0));
}
template <> __device__ __forceinline__ bf16_t bload<bf16_t>(__amdgpu_buffer_rsrc_t r, int voff, int soff) {
    return __builtin_amdgcn_raw_buffer_load_b16(r, voff, soff, 0);
}
// scaled value for the LDS store (BF16: scaled in FP32, rounded back)
template <class T, class S> __device__ __forceinline__ T scaled(T v, S s) { return v * s; }
template <> __device__ __forceinline__ bf16_t scaled<bf16_t, float>(bf16_t v, float s) {
    return s == 1.0f ? v : f2bf(bf2f(v) * s);
}

template <class T, int BK>
struct Slice {
    static constexpr int E = BK / 4;
    // row padding: 2 doubles, 4 floats, 8 bf16 (BF16 rows stay 16-byte aligned
    // for the 8-wide fragment reads)
    static constexpr int LDK = BK + (sizeof(T) == 8 ? 2 : (sizeof(T) == 4 ? 4 : 8));
    typedef typename MmaTraits<T>::scale_t S;
    T v[E];
    S scale;
    // Global loads of one slice.  Element (r, k) lies at P[r*ld + k] ("along
    // K": lane -> k = t % BK, rows t / BK + RS u) or at P[k*ld + r] ("along
    // M/N": lane -> r = t % 16 + 16 (t / 64), k = (t / 16) % 4 + 4 u; 16
    // consecutive r per row for coalescing, and a wave's LDS stores then fall
    // in 64 different banks).  Both layouts reduce to per-element byte offsets
    // base + u step for u below a count nv, so one set of loads serves both:
    // the staged values sit in the same registers whatever a chunk's layout,
    // and nothing forces the loads of one slice to complete before the MFMAs
    // of the previous one.
    __device__ __forceinline__ void load(const T* P, bool along_k, int ld, int r0, int rmax, int k0, int K, S s,
                                         int tid) {
        constexpr int RS = NTH / BK;
        constexpr int SH = RS == 8 ? 3 : (RS == 16 ? 4 : 5);
        static_assert((1 << SH) == RS, "rows per pass must be 8, 16 or 32");
        int base, step, nv;
        if (along_k) {
            const int k = tid % BK, r = tid / BK;
            base = ((r0 + r) * ld + k0 + k) * (int)sizeof(T);
            step = RS * ld * (int)sizeof(T);
            nv = k0 + k < K ? (rmax - r + RS - 1) >> SH : 0;
        } else {
            const int r = (tid & 15) + 16 * (tid >> 6), k = (tid >> 4) & 3;
            base = ((k0 + k) * ld + r0 + r) * (int)sizeof(T);
            step = 4 * ld * (int)sizeof(T);
            nv = r < rmax ? (K - k0 - k + 3) >> 2 : 0;
        }
        const __amdgpu_buffer_rsrc_t rs = make_rsrc(P);
        scale = s;
#pragma unroll
        for (int u = 0; u < E; ++u) v[u] = bload<T>(rs, u < nv ? base + u * step : kOutside, 0);
    }
    // LDS position of slice column k: FP32 / FP64 slices are stored k-permuted,
    // k -> E (k % 4) + k / 4, so that the values a lane feeds to its MFMA steps
    // q = 0 .. E-1 (k = 4 q + lane / 16) are contiguous and read as 16-byte
    // vectors; BF16 keeps k in order (its fragments are already 8 wide).
    static __device__ __forceinline__ int pos(int k) { return sizeof(T) == 2 ? k : E * (k & 3) + (k >> 2); }
    __device__ __forceinline__ void store_k(T* __restrict__ Sm, int tid) const {
        constexpr int RS = NTH / BK;
        const int k = tid % BK, r = tid / BK;
        const int pk = pos(k);
#pragma unroll
        for (int u = 0; u < E; ++u) Sm[(r + RS * u) * LDK + pk] = scaled(v[u], scale);
    }
    __device__ __forceinline__ void store_m(T* __restrict__ Sm, int tid) const {
        const int r = (tid & 15) + 16 * (tid >> 6), k = (tid >> 4) & 3;
        if constexpr (sizeof(T) == 2) {
#pragma unroll
            for (int u = 0; u < E; ++u) Sm[r * LDK + k + 4 * u] = scaled(v[u], scale);
        } else {
            // elements (r, k + 4 u), u = 0 .. E-1, land at E k + u: contiguous
            typedef T v4 __attribute__((ext_vector_type(16 / sizeof(T))));
            constexpr int W = 16 / sizeof(T);
            T* dst = &Sm[r * LDK + E * k];
#pragma unroll
            for (int h = 0; h < E / W; ++h) {
                v4 x;
#pragma unroll
                for (int w = 0; w < W; ++w) x[w] = scaled(v[h * W + w], scale);
                *(v4*)(dst + h * W) = x;
            }
        }
    }
};

// Where a GEMM finds its buffer table: a kernel argument (single plan), or
// an LDS copy of a plan's table (grouped launches); in both cases a buffer's
// base address is uniform over the work-group and kept in scalar registers.
struct ArgBufs {
    const Bufs& b;
    __device__ __forceinline__ void* get(int i) const { return b.p[i]; }
};
struct LdsBufs {
    const Bufs* b;   // in LDS
    __device__ __forceinline__ void* get(int i) const {
        const uint64_t v = (uint64_t)b->p[i];
        const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)v);
        const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)(v >> 32));
        return (void*)(((uint64_t)hi << 32) | lo);
    }
};

// Persistent grouped GEMM (the FP64 and BF16 instantiations; FP32 runs
// gemm_body_f32dma below).  Work-group w runs its task list
// [wg_off[w], wg_off[w+1]) (balanced on the host).  One software pipeline runs
// over the K slices of all its chunks and tasks: the next slice's global loads
// (possibly of the next task) are in flight while the MFMAs consume the current
// slice from LDS; a task's epilogue is written when its last slice has been
// consumed.
// Task, chunk and schedule lists are read-only during a launch: they are read
// through constant-address-space pointers, so that their uniform loads are
// scalar loads whatever the origin of the pointers (kernel arguments, or a
// plan table in memory for grouped launches).
template <class T> using cptr = const __attribute__((address_space(4))) T*;
template <class T> __device__ __forceinline__ cptr<T> as_const(const T* p) { return (cptr<T>)(uintptr_t)p; }
// element i of a constant-address-space array, copied word by word
template <class T> __device__ __forceinline__ T ldc(cptr<T> p, int64_t i) {
    static_assert(sizeof(T) % 4 == 0, "descriptor size");
    const __attribute__((address_space(4))) uint32_t* w = (const __attribute__((address_space(4))) uint32_t*)(p + i);
    T v;
    uint32_t* o = reinterpret_cast<uint32_t*>(&v);
#pragma unroll
    for (int k = 0; k < (int)(sizeof(T) / 4); ++k) o[k] = w[k];
    return v;
}

template <class T, class TC, int BK, class BS>
__device__ __forceinline__ void gemm_body(const BS bufs, const GemmTask* __restrict__ tasks_g,
                                          const GemmChunk* __restrict__ chunks_g, const Sched& sc, int wg, int nwg) {
    const cptr<GemmTask> tasks = as_const(tasks_g);
    const cptr<GemmChunk> chunks = as_const(chunks_g);
    const cptr<int32_t> wg_off = as_const(sc.wg_off);
    typedef typename MmaTraits<T>::acc_t acc_t;
    typedef Slice<T, BK> SL;
    constexpr int LDK = SL::LDK;
    __shared__ __attribute__((aligned(16))) T As[2][TM * LDK];
    __shared__ __attribute__((aligned(16))) T Bs[2][TN * LDK];
    const int tid = threadIdx.x;
    // The wave index is uniform across a wave.  The FP32 and BF16 bodies keep
    // it in a scalar register: the quadrant tests below become scalar branches
    // rather than exec-mask updates, and the next slice's global loads stay in
    // flight over the MFMAs instead of being waited for at the branch join.
    // The FP64 body (no such wait) needs the vector registers more and keeps
    // it per lane.
    const int wave = sizeof(T) == 8 ? tid >> 6 : __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;   // wave quadrant
    const int fr = lane & 15, fk = lane >> 4;
    int ti = wg_off[wg];
    const int hi = wg_off[wg + 1];
    acc_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = acc_t{0, 0, 0, 0};
    SL ra, rb;
    auto load = [&](const GemmTask& t, const GemmChunk& ch, int k0) {
        const T* A = (const T*)bufs.get(ch.a_buf) + ch.a_off;
        const T* B = (const T*)bufs.get(ch.b_buf) + ch.b_off;
        typedef typename MmaTraits<T>::scale_t S;
        const S alpha = (S)ch.alpha;
        ra.load(A, !ch.a_trans, ch.lda, t.m0, t.mt, k0, ch.K, alpha, tid);
        rb.load(B, ch.b_trans, ch.ldb, t.n0, t.nt, k0, ch.K, S(1), tid);
    };
    auto store = [&](const GemmChunk& ch, int buf) {
        if (!ch.a_trans) ra.store_k(As[buf], tid);
        else ra.store_m(As[buf], tid);
        if (!ch.b_trans) rb.store_m(Bs[buf], tid);
        else rb.store_k(Bs[buf], tid);
    };
    auto epilogue = [&](const GemmTask& t) {
        TC* C = (TC*)bufs.get(t.c_buf) + t.c_off;
        const int64_t ldc = t.c_local ? TN : t.ldc;
        const int64_t base = t.c_local ? 0 : (int64_t)t.m0 * t.ldc + t.n0;
        TC old[2][2][4];
        if (t.beta) {   // all reads in flight before the first use
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm + a * 16 + MmaTraits<T>::row(lane, r);
                        const int col = wn + b * 16 + (lane & 15);
                        const bool in = row < t.mt && col < t.nt;
                        old[a][b][r] = C[in ? base + (int64_t)row * ldc + col : base];
                    }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm + a * 16 + MmaTraits<T>::row(lane, r);
                    const int col = wn + b * 16 + (lane & 15);
                    if (row < t.mt && col < t.nt) {
                        double v = (double)acc[a][b][r];
                        if (t.beta) v += from_out<TC>(old[a][b][r]);
                        C[base + (int64_t)row * ldc + col] = to_out<TC>(v);
                    }
                    acc[a][b][r] = 0;
                }
    };
    if (ti < hi) {
        GemmTask tk = ldc(tasks, ti);
        int c = tk.chunk_begin;
        GemmChunk ch = ldc(chunks, c);
        int k0 = 0;
        // descriptors of this work-group's next task, fetched a whole task ahead
        int pti = ti + 1;
        GemmTask ptk = tk;
        GemmChunk pch = ch;
        if (pti < hi) {
            ptk = ldc(tasks, pti);
            pch = ldc(chunks, ptk.chunk_begin);
        }
        load(tk, ch, 0);
        store(ch, 0);
        __syncthreads();
        int buf = 0;
        while (true) {
            // successor slice: same chunk, next chunk, or the next task's first chunk
            GemmTask ntk = tk;
            int nc = c, nk0 = k0 + BK;
            GemmChunk nch = ch;
            bool newtask = false, more = true;
            if (nk0 >= ch.K) {
                nk0 = 0;
                nc = c + 1;
                if (nc < tk.chunk_end) {
                    nch = ldc(chunks, nc);
                } else {
                    newtask = true;
                    more = pti < hi;
                    ntk = ptk;
                    nc = ptk.chunk_begin;
                    nch = pch;
                }
            }
            if (more) load(ntk, nch, nk0);   // global loads in flight during the MFMAs
            const T* Ab = As[buf];
            const T* Bb = Bs[buf];
            typedef typename MmaTraits<T>::frag_t F;
            constexpr int KS = MmaTraits<T>::KS, NS = BK / KS;
            // a lane's fragment: row fr of the 16-row block, k = s KS + fk (one
            // element) or s KS + 8 fk .. +7 (BF16, one 16-byte read)
            auto frag = [&](const T* S, int row, int s) -> F {
                if constexpr (sizeof(T) == 2) return *(const F*)&S[row * LDK + s * KS + 8 * fk];
                else return S[row * LDK + s * KS + fk];
            };
            // FP64 / FP32: all fragments of the slice first (k-permuted rows: a
            // lane's NS values are contiguous, read as 16-byte vectors), then the
            // MFMAs back to back; BF16 (8 VGPRs of fragments per step): one step
            // at a time
            constexpr int NF = sizeof(T) == 2 ? 1 : NS;
            F av[NF][2], bv[NF][2];
            auto fetch = [&](int q) {
#pragma unroll
                for (int a = 0; a < 2; ++a) av[q % NF][a] = frag(Ab, wm + a * 16 + fr, q);
#pragma unroll
                for (int b = 0; b < 2; ++b) bv[q % NF][b] = frag(Bb, wn + b * 16 + fr, q);
            };
            if constexpr (NF == NS && sizeof(T) == 2) {
#pragma unroll
                for (int q = 0; q < NS; ++q) fetch(q);
            } else if constexpr (NF == NS) {
                typedef T v4 __attribute__((ext_vector_type(16 / sizeof(T))));
                constexpr int W = 16 / sizeof(T);
#pragma unroll
                for (int a = 0; a < 2; ++a) {
                    const T* pa = &Ab[(wm + a * 16 + fr) * LDK + NS * fk];
                    const T* pb = &Bb[(wn + a * 16 + fr) * LDK + NS * fk];
#pragma unroll
                    for (int h = 0; h < NS / W; ++h) {
                        const v4 xa = *(const v4*)(pa + h * W);
                        const v4 xb = *(const v4*)(pb + h * W);
#pragma unroll
                        for (int w = 0; w < W; ++w) {
                            av[h * W + w][a] = xa[w];
                            bv[h * W + w][a] = xb[w];
                        }
                    }
                }
            }
            // MFMAs of 16 x 16 blocks that lie wholly outside the tile, and
            // K steps past the chunk's end, are skipped (wave-uniform tests):
            // ragged sector blocks cost what they contain.
            const int kv = ch.K - k0;
            const bool am1 = wm + 16 < tk.mt, bm1 = wn + 16 < tk.nt;
            // Full blocks: the next slice goes into the other LDS buffer halfway
            // through the MFMAs, whose queue then covers the stores.
            bool stored = false;
            if (kv >= BK && am1 && bm1) {
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    if (NF != NS) fetch(q);
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b)
                            acc[a][b] = MmaTraits<T>::mma(av[q % NF][a], bv[q % NF][b], acc[a][b]);
                    if (q == NS / 2 - 1 && more) {
                        store(nch, buf ^ 1);
                        stored = true;
                    }
                }
            } else if (wm < tk.mt && wn < tk.nt) {
#pragma unroll
                for (int q = 0; q < NS; ++q) {
                    if (KS * q < kv) {
                        if (NF != NS) fetch(q);
                        const int f = q % NF;
                        acc[0][0] = MmaTraits<T>::mma(av[f][0], bv[f][0], acc[0][0]);
                        if (bm1) acc[0][1] = MmaTraits<T>::mma(av[f][0], bv[f][1], acc[0][1]);
                        if (am1) acc[1][0] = MmaTraits<T>::mma(av[f][1], bv[f][0], acc[1][0]);
                        if (am1 && bm1) acc[1][1] = MmaTraits<T>::mma(av[f][1], bv[f][1], acc[1][1]);
                    }
                }
            }
            if (newtask) {
                epilogue(tk);
                if (more) {
                    ti = pti;
                    pti = ti + 1;
                    if (pti < hi) {
                        ptk = ldc(tasks, pti);
                        pch = ldc(chunks, ptk.chunk_begin);
                    }
                }
            }
            if (more && !stored) store(nch, buf ^ 1);
            __syncthreads();
            if (!more) break;
            tk = ntk;
            c = nc;
            k0 = nk0;
            ch = nch;
            buf ^= 1;
        }
    }
    // tasks without chunks: clear their tile (beta = 0) or leave it (beta = 1)
    for (int t = sc.nfull + wg; t < sc.ntasks; t += nwg) {
        const GemmTask z = ldc(tasks, t);
        if (z.beta) continue;
        TC* C = (TC*)bufs.get(z.c_buf) + z.c_off;
        const int64_t ldc = z.c_local ? TN : z.ldc;
        const int64_t base = z.c_local ? 0 : (int64_t)z.m0 * z.ldc + z.n0;
        for (int e = tid; e < TM * TN; e += NTH) {
            const int r = e / TN, q = e % TN;
            if (r < z.mt && q < z.nt) C[base + (int64_t)r * ldc + q] = (TC)0;
        }
    }
}

// FP32 grouped GEMM with direct-to-LDS loads.  Each K slice (32 deep) of a
// 64-row operand tile is 8 KB, written into LDS by 16-byte buffer loads that
// bypass the registers (two per wave and operand); each load of a wave fills
// 1 KB of LDS in lane order, so the layout is chosen through which global
// chunk each lane fetches:
//  - K contiguous: rows of 32 k (128 B); 16-byte chunk c of row r sits at
//    position c ^ swz_k(r) of its row;
//  - M (or N) contiguous: k-rows of 64 m (256 B); chunk g (4 rows) of k-row kr
//    sits at position g ^ swz_m(kr).
// The swizzles keep the fragment reads (16-byte reads of one row's chunk, or
// 4-byte reads down a k-column) on distinct banks.  MFMA step q of lane group
// fk takes k = 16 (q / 4) + 4 fk + q % 4 (any one-to-one map works when both
// operands use it): a K-contiguous fragment is one chunk per half slice, and
// a slice whose chunk ends in its first half skips the second half's steps.
// One barrier per slice: after it, the next slice's loads go into the other
// buffer, which every wave has finished reading.
// Bounds: chunks past the operand's K or rows are fetched with an offset past
// the resource range and land as zeros; the range is the tile's extent, so a
// chunk that crosses it gets zeros beyond it without a memory access.  Values
// past K that a K-contiguous chunk carries from inside the block are replaced
// by zero after the fragment read; values of rows past the tile's edge only
// reach output rows that are not written.
__device__ __forceinline__ int swz_k(int r) { return (r ^ (r >> 3)) & 7; }
__device__ __forceinline__ int swz_m(int kr) { return 4 * ((kr >> 2) & 3); }
typedef __attribute__((address_space(3))) void* lds_ptr_t;
// this wave's two 1 KB pieces of one operand's slice into the LDS tile `dst`
// (2048 floats); `P` is the operand block, rows r0 .. r0 + rmax - 1 of it
__device__ __forceinline__ void dma_slice(float* dst, const float* P, bool along_k, int ld, int r0, int rmax,
                                          int k0, int K, int wave, int lane) {
    const int ext = along_k ? ((r0 + rmax - 1) * ld + K) * 4 : ((K - 1) * ld + r0 + rmax) * 4;
    // uniform over the wave: kept in a scalar register, as the resource must be
    const int range = __builtin_amdgcn_readfirstlane(ext < 0 ? 0 : (ext > kRecords ? kRecords : ext));
    const __amdgpu_buffer_rsrc_t rs =
        __builtin_amdgcn_make_buffer_rsrc(const_cast<float*>(P), (short)0, range, 0x00020000);
#pragma unroll
    for (int i = 0; i < 2; ++i) {
        int off, lds;
        if (along_k) {
            const int R0 = 16 * wave + 8 * i, r = R0 + (lane >> 3);
            const int c = (lane & 7) ^ swz_k(r);
            const int o = ((r0 + r) * ld + k0 + 4 * c) * 4;
            off = (r < rmax) & (k0 + 4 * c < K) ? o : kOutside;
            lds = R0 * 32;
        } else {
            const int K0 = 8 * wave + 4 * i, kr = K0 + (lane >> 4);
            const int g = (lane & 15) ^ swz_m(kr);
            const int o = ((k0 + kr) * ld + r0 + 4 * g) * 4;
            off = (k0 + kr < K) & (4 * g < rmax) ? o : kOutside;
            lds = K0 * 64;
        }
        __builtin_amdgcn_raw_ptr_buffer_load_lds(rs, (lds_ptr_t)(dst + lds), 16, off, 0, 0, 0);
    }
}
// one operand's fragments (two 16-row blocks, 8 k each) of the slice in `src`
__device__ __forceinline__ void frag_read(float (&f)[2][8], const float* src, bool along_k, int w0, int fr, int fk) {
    if (along_k) {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int r = w0 + 16 * a + fr;
#pragma unroll
            for (int h = 0; h < 2; ++h) {
                const int slot = (4 * h + fk) ^ swz_k(r);
                const f4_t v = *(const f4_t*)&src[r * 32 + slot * 4];
#pragma unroll
                for (int j = 0; j < 4; ++j) f[a][4 * h + j] = v[j];
            }
        }
    } else {
#pragma unroll
        for (int a = 0; a < 2; ++a) {
            const int r = w0 + 16 * a + fr;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const int kr = 16 * (q >> 2) + 4 * fk + (q & 3);
                const int slot = (r >> 2) ^ swz_m(kr);
                f[a][q] = src[kr * 64 + slot * 4 + (r & 3)];
            }
        }
    }
}

template <class TC, class BS>
__device__ __forceinline__ void gemm_body_f32dma(const BS bufs, const GemmTask* __restrict__ tasks_g,
                                                 const GemmChunk* __restrict__ chunks_g, const Sched& sc, int wg,
                                                 int nwg) {
    const cptr<GemmTask> tasks = as_const(tasks_g);
    const cptr<GemmChunk> chunks = as_const(chunks_g);
    const cptr<int32_t> wg_off = as_const(sc.wg_off);
    typedef MmaTraits<float> MT;
    // two buffers per operand, as separate objects so that the compiler can tell
    // the loads into one from the reads of the other
    __shared__ __attribute__((aligned(16))) float A0[2048], A1[2048], B0[2048], B1[2048];
    const int tid = threadIdx.x;
    const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
    const int lane = tid & 63;
    const int wm = (wave >> 1) * 32, wn = (wave & 1) * 32;   // wave quadrant
    const int fr = lane & 15, fk = lane >> 4;
    int ti = wg_off[wg];
    const int hi = wg_off[wg + 1];
    f4_t acc[2][2];
#pragma unroll
    for (int a = 0; a < 2; ++a)
#pragma unroll
        for (int b = 0; b < 2; ++b) acc[a][b] = f4_t{0, 0, 0, 0};
    auto ptr_a = [&](const GemmChunk& ch) { return (const float*)bufs.get(ch.a_buf) + ch.a_off; };
    auto ptr_b = [&](const GemmChunk& ch) { return (const float*)bufs.get(ch.b_buf) + ch.b_off; };
    auto dma = [&](float* da, float* db, const GemmTask& t, const GemmChunk& ch, const float* pa, const float* pb,
                   int k0) {
        dma_slice(da, pa, !ch.a_trans, ch.lda, t.m0, t.mt, k0, ch.K, wave, lane);
        dma_slice(db, pb, ch.b_trans, ch.ldb, t.n0, t.nt, k0, ch.K, wave, lane);
    };
    auto compute = [&](const float* sa, const float* sb, const GemmTask& t, const GemmChunk& ch, int k0) {
        if (!(wm < t.mt && wn < t.nt)) return;
        const int kv = ch.K - k0;
        const bool am1 = wm + 16 < t.mt, bm1 = wn + 16 < t.nt;
        const bool ak = !ch.a_trans, bk = ch.b_trans;
        float fa[2][8], fb[2][8];
        frag_read(fa, sa, ak, wm, fr, fk);
        frag_read(fb, sb, bk, wn, fr, fk);
        if (kv < 32 && (ak || bk)) {
            const int lim = kv - 4 * fk;
#pragma unroll
            for (int q = 0; q < 8; ++q) {
                const bool ok = 16 * (q >> 2) + (q & 3) < lim;
#pragma unroll
                for (int i = 0; i < 2; ++i) {
                    if (ak) fa[i][q] = ok ? fa[i][q] : 0.0f;
                    if (bk) fb[i][q] = ok ? fb[i][q] : 0.0f;
                }
            }
        }
        const float alpha = (float)ch.alpha;
        if (alpha != 1.0f) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
#pragma unroll
                for (int i = 0; i < 2; ++i) fa[i][q] *= alpha;
        }
        const int nq = kv > 16 ? 8 : 4;
        if (am1 && bm1) {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nq) {
#pragma unroll
                    for (int a = 0; a < 2; ++a)
#pragma unroll
                        for (int b = 0; b < 2; ++b) acc[a][b] = MT::mma(fa[a][q], fb[b][q], acc[a][b]);
                }
        } else {
#pragma unroll
            for (int q = 0; q < 8; ++q)
                if (q < nq) {
                    acc[0][0] = MT::mma(fa[0][q], fb[0][q], acc[0][0]);
                    if (bm1) acc[0][1] = MT::mma(fa[0][q], fb[1][q], acc[0][1]);
                    if (am1) acc[1][0] = MT::mma(fa[1][q], fb[0][q], acc[1][0]);
                }
        }
    };
    auto epilogue = [&](const GemmTask& t) {
        TC* C = (TC*)bufs.get(t.c_buf) + t.c_off;
        const int64_t ldc = t.c_local ? TN : t.ldc;
        const int64_t base = t.c_local ? 0 : (int64_t)t.m0 * t.ldc + t.n0;
        TC old[2][2][4];
        if (t.beta) {
#pragma unroll
            for (int a = 0; a < 2; ++a)
#pragma unroll
                for (int b = 0; b < 2; ++b)
#pragma unroll
                    for (int r = 0; r < 4; ++r) {
                        const int row = wm + a * 16 + MT::row(lane, r);
                        const int col = wn + b * 16 + (lane & 15);
                        const bool in = row < t.mt && col < t.nt;
                        old[a][b][r] = C[in ? base + (int64_t)row * ldc + col : base];
                    }
        }
#pragma unroll
        for (int a = 0; a < 2; ++a)
#pragma unroll
            for (int b = 0; b < 2; ++b)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int row = wm + a * 16 + MT::row(lane, r);
                    const int col = wn + b * 16 + (lane & 15);
                    if (row < t.mt && col < t.nt) {
                        double v = (double)acc[a][b][r];
                        if (t.beta) v += from_out<TC>(old[a][b][r]);
                        C[base + (int64_t)row * ldc + col] = to_out<TC>(v);
                    }
                    acc[a][b][r] = 0;
                }
    };
    if (ti < hi) {
        GemmTask tk = ldc(tasks, ti);
        int c = tk.chunk_begin;
        GemmChunk ch = ldc(chunks, c);
        const float* pa = ptr_a(ch);
        const float* pb = ptr_b(ch);
        int k0 = 0;
        int pti = ti + 1;
        GemmTask ptk = tk;
        if (pti < hi) ptk = ldc(tasks, pti);
        dma(A0, B0, tk, ch, pa, pb, 0);
        // one slice: wait for its loads, start the successor's loads into the
        // other buffers, then the MFMAs on this one
        auto step = [&](const float* sa, const float* sb, float* na, float* nb) -> bool {
            GemmTask ntk = tk;
            int nc = c, nk0 = k0 + 32;
            GemmChunk nch = ch;
            const float* npa = pa;
            const float* npb = pb;
            bool newtask = false, more = true;
            if (nk0 >= ch.K) {
                nk0 = 0;
                nc = c + 1;
                if (nc < tk.chunk_end) {
                    nch = ldc(chunks, nc);
                } else {
                    newtask = true;
                    more = pti < hi;
                    if (more) {
                        ntk = ptk;
                        nc = ntk.chunk_begin;
                        nch = ldc(chunks, nc);
                    }
                }
                npa = ptr_a(nch);
                npb = ptr_b(nch);
            }
            __builtin_amdgcn_s_waitcnt(0x0F70);   // vmcnt(0): this wave's loads of the slice are in LDS
            __syncthreads();                       // everyone's are; the other buffers are free
            if (more) dma(na, nb, ntk, nch, npa, npb, nk0);
            compute(sa, sb, tk, ch, k0);
            if (newtask) {
                epilogue(tk);
                if (more) {
                    ti = pti;
                    pti = ti + 1;
                    if (pti < hi) ptk = ldc(tasks, pti);
                }
            }
            tk = ntk;
            c = nc;
            ch = nch;
            pa = npa;
            pb = npb;
            k0 = nk0;
            return more;
        };
        while (step(A0, B0, A1, B1) && step(A1, B1, A0, B0)) {
        }
    }
    // tasks without chunks: clear their tile (beta = 0) or leave it (beta = 1)
    for (int t = sc.nfull + wg; t < sc.ntasks; t += nwg) {
        const GemmTask z = ldc(tasks, t);
        if (z.beta) continue;
        TC* C = (TC*)bufs.get(z.c_buf) + z.c_off;
        const int64_t ldc = z.c_local ? TN : z.ldc;
        const int64_t base = z.c_local ? 0 : (int64_t)z.m0 * z.ldc + z.n0;
        for (int e = tid; e < TM * TN; e += NTH) {
            const int r = e / TN, q = e % TN;
            if (r < z.mt && q < z.nt) C[base + (int64_t)r * ldc + q] = (TC)0;
        }
    }
}

// The same body under three names, so that profiles separate the two
// H_eff phases from the renormalisation and prediction GEMMs.
// FP32 products use the direct-to-LDS body, the other precisions the staged one
template <class T, class TC, int BK, class BS>
__device__ __forceinline__ void any_body(const BS bufs, const GemmTask* t, const GemmChunk* c, const Sched& s, int wg,
                                         int nwg) {
    if constexpr (sizeof(T) == 4) gemm_body_f32dma<TC>(bufs, t, c, s, wg, nwg);
    else gemm_body<T, TC, BK>(bufs, t, c, s, wg, nwg);
}
template <class T, class TC, int BK>
__global__ void __launch_bounds__(NTH, 4) k_gemm(Bufs b, const GemmTask* t, const GemmChunk* c, Sched s) {
    any_body<T, TC, BK>(ArgBufs{b}, t, c, s, blockIdx.x, gridDim.x);
}
template <class T, class TC, int BK>
__global__ void __launch_bounds__(NTH, 4) k_heff_z(Bufs b, const GemmTask* t, const GemmChunk* c, Sched s) {
    any_body<T, TC, BK>(ArgBufs{b}, t, c, s, blockIdx.x, gridDim.x);
}
template <class T, class TC, int BK>
__global__ void __launch_bounds__(NTH, 4) k_heff_y(Bufs b, const GemmTask* t, const GemmChunk* c, Sched s) {
    any_body<T, TC, BK>(ArgBufs{b}, t, c, s, blockIdx.x, gridDim.x);
}

// Grouped launch over several plans (independent solves advanced together):
// work-group g runs plan p, wg_prefix[p] <= g < wg_prefix[p + 1], as its
// work-group g - wg_prefix[p], with that plan's buffers and schedule.
__device__ __forceinline__ int plan_of(const int32_t* __restrict__ prefix, int nplans, int g) {
    int p = 0;
    while (p + 1 < nplans && prefix[p + 1] <= g) ++p;
    // uniform over the work-group: in a scalar register, so that the plan's
    // descriptors are scalar loads as in the single-plan kernels
    return __builtin_amdgcn_readfirstlane(p);
}
template <class T, class TC, int BK>
__device__ __forceinline__ void multi_body(const PlanDesc* __restrict__ plans, const int32_t* __restrict__ prefix,
                                           int nplans) {
    const int p = plan_of(prefix, nplans, blockIdx.x);
    // the buffer table stays in memory (a local copy indexed by the chunks'
    // buffer numbers would live in scratch)
    // the plan's fields, each a scalar load at its offset
    const uintptr_t base = (uintptr_t)(plans + p);
    auto u64 = [&](size_t off) { return *(const __attribute__((address_space(4))) uint64_t*)(base + off); };
    auto i32 = [&](size_t off) { return *(const __attribute__((address_space(4))) int32_t*)(base + off); };
    constexpr size_t bo = offsetof(PlanDesc, bufs), so = offsetof(PlanDesc, sc);
    __shared__ Bufs tab;
    if (threadIdx.x < kMaxBufs) tab.p[threadIdx.x] = (void*)u64(bo + 8 * threadIdx.x);
    __syncthreads();
    const LdsBufs b{&tab};
    Sched sc;
    sc.wg_off = (const int32_t*)u64(so + offsetof(Sched, wg_off));
    sc.nwg = i32(so + offsetof(Sched, nwg));
    sc.nfull = i32(so + offsetof(Sched, nfull));
    sc.ntasks = i32(so + offsetof(Sched, ntasks));
    any_body<T, TC, BK>(b, (const GemmTask*)u64(offsetof(PlanDesc, tasks)),
                        (const GemmChunk*)u64(offsetof(PlanDesc, chunks)), sc, blockIdx.x - prefix[p],
                        prefix[p + 1] - prefix[p]);
}
template <class T, class TC, int BK>
__global__ void __launch_bounds__(NTH, 4) k_multi_gemm(const PlanDesc* p, const int32_t* x, int n) {
    multi_body<T, TC, BK>(p, x, n);
}
template <class T, class TC, int BK>
__global__ void __launch_bounds__(NTH, 4) k_multi_heff_z(const PlanDesc* p, const int32_t* x, int n) {
    multi_body<T, TC, BK>(p, x, n);
}
template <class T, class TC, int BK>
__global__ void __launch_bounds__(NTH, 4) k_multi_heff_y(const PlanDesc* p, const int32_t* x, int n) {
    multi_body<T, TC, BK>(p, x, n);
}

int gemm_multi(Ctx* c, int ab, int cp, const PlanDesc* plans, const int32_t* prefix, int nplans, int total_wg,
               int kind) {
    if (nplans <= 0 || total_wg <= 0) return 0;
    dim3 grid(total_wg), block(NTH);
#define MULTI(T, TC, BK)                                                                                   \
    do {                                                                                                   \
        if (kind == GK_HEFF_Z)                                                                             \
            hipLaunchKernelGGL((k_multi_heff_z<T, TC, BK>), grid, block, 0, c->stream, plans, prefix, nplans); \
        else if (kind == GK_HEFF_Y)                                                                        \
            hipLaunchKernelGGL((k_multi_heff_y<T, TC, BK>), grid, block, 0, c->stream, plans, prefix, nplans); \
        else                                                                                               \
            hipLaunchKernelGGL((k_multi_gemm<T, TC, BK>), grid, block, 0, c->stream, plans, prefix, nplans);  \
    } while (0)
    if (ab == P_F64 && cp == P_F64) MULTI(double, double, 16);
    else if (ab == P_F32 && cp == P_F32) MULTI(float, float, 32);
    else if (ab == P_BF16 && cp == P_F32) MULTI(bf16_t, float, 32);
    else if (ab == P_BF16 && cp == P_BF16) MULTI(bf16_t, bf16_t, 32);
    else {
        c->err = "unsupported GEMM precision combination";
        return 1;
    }
#undef MULTI
    LAUNCHCHK(c);
    return 0;
}

int gemm(Ctx* c, int ab, int cp, void* const* bufs, const GemmTask* tasks, const Sched& sc,
         const GemmChunk* chunks, int kind, int ev_start, int ev_stop) {
    const int ntasks = sc.ntasks;
    if (ntasks <= 0) return 0;
    Bufs b;
    for (int i = 0; i < kMaxBufs; ++i) b.p[i] = bufs[i];
    const dim3 pgrid(std::max(1, sc.nwg)), block(NTH);
    hipEvent_t e0 = ev_start >= 0 ? c->ev[ev_start] : nullptr, e1 = ev_stop >= 0 ? c->ev[ev_stop] : nullptr;
    auto go = [&](auto kern) {
        if (e0 || e1)
            hipExtLaunchKernelGGL(kern, pgrid, block, 0, c->stream, e0, e1, 0, b, tasks, chunks, sc);
        else
            hipLaunchKernelGGL(kern, pgrid, block, 0, c->stream, b, tasks, chunks, sc);
    };
    if (ab == P_F64 && cp == P_F64) {
        if (kind == GK_HEFF_Z) go(k_heff_z<double, double, 16>);
        else if (kind == GK_HEFF_Y) go(k_heff_y<double, double, 16>);
        else go(k_gemm<double, double, 16>);
    } else if (ab == P_F32 && cp == P_F32) {
        if (kind == GK_HEFF_Z) go(k_heff_z<float, float, 32>);
        else if (kind == GK_HEFF_Y) go(k_heff_y<float, float, 32>);
        else go(k_gemm<float, float, 32>);
    } else if (ab == P_BF16 && cp == P_F32) {
        if (kind == GK_HEFF_Z) go(k_heff_z<bf16_t, float, 32>);
        else if (kind == GK_HEFF_Y) go(k_heff_y<bf16_t, float, 32>);
        else go(k_gemm<bf16_t, float, 32>);
    } else if (ab == P_BF16 && cp == P_BF16) {
        if (kind == GK_HEFF_Z) go(k_heff_z<bf16_t, bf16_t, 32>);
        else if (kind == GK_HEFF_Y) go(k_heff_y<bf16_t, bf16_t, 32>);
        else go(k_gemm<bf16_t, bf16_t, 32>);
    } else {
        c->err = "unsupported GEMM precision combination";
        return 1;
    }
    LAUNCHCHK(c);
    return 0;
}

// ------------------------------------------------------ split-K reduction
// Block (task, y) sums elements [256 y, 256 y + 256) of one tile over its
// slots in a fixed order (four interleaved partial sums, then combined), so
// results are deterministic and many loads are in flight per thread.
template <class TC>
__device__ __forceinline__ void reduce_body(const Bufs& bufs, const RedTask& tk) {
    const int e = blockIdx.y * 256 + threadIdx.x;
    const int r = e / TN, c = e % TN;
    if (r >= tk.mt || c >= tk.nt) return;
    const TC* P = (const TC*)bufs.p[kPartialBuf] + (int64_t)tk.slot0 * TM * TN + e;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0, s3 = 0.0;
    int q = 0;
    for (; q + 4 <= tk.nslots; q += 4) {
        s0 += (double)P[(int64_t)q * TM * TN];
        s1 += (double)P[(int64_t)(q + 1) * TM * TN];
        s2 += (double)P[(int64_t)(q + 2) * TM * TN];
        s3 += (double)P[(int64_t)(q + 3) * TM * TN];
    }
    for (; q < tk.nslots; ++q) s0 += (double)P[(int64_t)q * TM * TN];
    double s = (s0 + s1) + (s2 + s3);
    TC* d = (TC*)bufs.p[tk.dst_buf] + tk.dst_off + (int64_t)r * tk.ld + c;
    if (tk.beta) s += (double)*d;
    *d = (TC)s;
}
template <class TC>
__global__ void __launch_bounds__(256) k_gemm_reduce(Bufs bufs, const RedTask* __restrict__ tasks) {
    reduce_body<TC>(bufs, tasks[blockIdx.x]);
}
// reductions of several plans: block x is reduction x - prefix[p] of plan p
template <class TC>
__global__ void __launch_bounds__(256) k_gemm_reduce_multi(const RedDesc* __restrict__ plans,
                                                           const int32_t* __restrict__ prefix, int nplans) {
    const int p = plan_of(prefix, nplans, blockIdx.x);
    reduce_body<TC>(*reinterpret_cast<const Bufs*>(plans[p].bufs), plans[p].reds[blockIdx.x - prefix[p]]);
}

int gemm_reduce_multi(Ctx* c, int cp, const RedDesc* plans, const int32_t* prefix, int nplans, int total) {
    if (nplans <= 0 || total <= 0) return 0;
    dim3 grid(total, TM * TN / 256);
    if (cp == P_F64)
        hipLaunchKernelGGL(k_gemm_reduce_multi<double>, grid, dim3(256), 0, c->stream, plans, prefix, nplans);
    else if (cp == P_F32)
        hipLaunchKernelGGL(k_gemm_reduce_multi<float>, grid, dim3(256), 0, c->stream, plans, prefix, nplans);
    else {
        c->err = "split-K reduction supports FP64 and FP32 outputs";
        return 1;
    }
    LAUNCHCHK(c);
    return 0;
}

int gemm_reduce(Ctx* c, int cp, void* const* bufs, const RedTask* tasks, int ntasks) {
    if (ntasks <= 0) return 0;
    Bufs b;
    for (int i = 0; i < kMaxBufs; ++i) b.p[i] = bufs[i];
    if (cp == P_F64)
        hipLaunchKernelGGL(k_gemm_reduce<double>, dim3(ntasks, TM * TN / 256), dim3(256), 0, c->stream, b, tasks);
    else if (cp == P_F32)
        hipLaunchKernelGGL(k_gemm_reduce<float>, dim3(ntasks, TM * TN / 256), dim3(256), 0, c->stream, b, tasks);
    else {
        c->err = "split-K reduction supports FP64 and FP32 outputs";
        return 1;
    }
    LAUNCHCHK(c);
    return 0;
}

// ====================================================== linear combination
struct DBufs {
    double* p[kMaxBufs];
};

// One 32 x 32 tile of D = sum_t coef_t op(S_t) per work-group; a thread owns
// the elements e = tid + 256 u (row e / 32, column e % 32), so that a wave
// reads two 32-element rows of a plain source.  A transposed source is read
// along its own contiguous dimension and turned round in LDS.  Each element
// sums its terms in term order.
__global__ void __launch_bounds__(256) k_lincomb(DBufs bufs, const LcTask* __restrict__ tasks,
                                                 const LcTerm* __restrict__ terms) {
    __shared__ double T[kLcTile][kLcTile + 1];
    const LcTask tk = tasks[blockIdx.x];
    const int tid = threadIdx.x;
    double acc[4] = {0, 0, 0, 0};
    for (int t = tk.t_begin; t < tk.t_end; ++t) {
        const LcTerm L = terms[t];
        const double* S = L.ident ? nullptr : bufs.p[L.buf] + L.src_off;
        if (L.trans && !L.ident) {
            __syncthreads();   // the previous transposed term's readers are done
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + 256 * u, rr = e & 31, cc = e >> 5;
                T[cc][rr] = rr < tk.mt && cc < tk.nt ? S[(int64_t)(tk.c0 + cc) * L.ld + tk.r0 + rr] : 0.0;
            }
            __syncthreads();
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + 256 * u, r = e >> 5, c = e & 31;
                acc[u] += L.coef * T[c][r];
            }
        } else {
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                const int e = tid + 256 * u, r = e >> 5, c = e & 31;
                if (r >= tk.mt || c >= tk.nt) continue;
                const double v = L.ident ? (tk.r0 + r == tk.c0 + c ? 1.0 : 0.0)
                                         : S[(int64_t)(tk.r0 + r) * L.ld + tk.c0 + c];
                acc[u] += L.coef * v;
            }
        }
    }
    double* D = bufs.p[tk.buf] + tk.dst_off;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int e = tid + 256 * u, r = e >> 5, c = e & 31;
        if (r < tk.mt && c < tk.nt) D[(int64_t)(tk.r0 + r) * tk.ld + tk.c0 + c] = acc[u];
    }
}

int lincomb(Ctx* c, double* const* bufs, const LcTask* tasks, int ntasks, const LcTerm* terms) {
    if (ntasks <= 0) return 0;
    DBufs b;
    for (int i = 0; i < kMaxBufs; ++i) b.p[i] = i < 2 ? bufs[i] : nullptr;
    hipLaunchKernelGGL(k_lincomb, dim3(ntasks), dim3(256), 0, c->stream, b, tasks, terms);
    LAUNCHCHK(c);
    return 0;
}

// ========================================================== H_eff diagonal
__global__ void __launch_bounds__(256) k_diag(DBufs bufs, const DiagTask* __restrict__ tasks,
                                              const DiagTerm* __restrict__ terms) {
    const DiagTask tk = tasks[blockIdx.x];
    const int tid = threadIdx.x;
    const int r = tid >> 3, c4 = (tid & 7) * 4;
    double acc[4] = {0, 0, 0, 0};
    for (int t = tk.t_begin; t < tk.t_end; ++t) {
        const DiagTerm d = terms[t];
        if (r >= tk.mt) continue;
        double a = d.a_ident ? 1.0 : bufs.p[d.a_buf][d.a_off + (int64_t)(tk.r0 + r) * d.a_step];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
            if (c4 + u >= tk.nt) continue;
            double b = d.b_ident ? 1.0 : bufs.p[d.b_buf][d.b_off + (int64_t)(tk.c0 + c4 + u) * d.b_step];
            acc[u] += d.coef * a * b;
        }
    }
    double* D = bufs.p[2] + tk.d_off;
#pragma unroll
    for (int u = 0; u < 4; ++u)
        if (r < tk.mt && c4 + u < tk.nt) D[(int64_t)(tk.r0 + r) * tk.ld + tk.c0 + c4 + u] = acc[u];
}

int diag(Ctx* c, double* const* bufs, const DiagTask* tasks, int ntasks, const DiagTerm* terms) {
    if (ntasks <= 0) return 0;
    DBufs b;
    for (int i = 0; i < kMaxBufs; ++i) b.p[i] = i < 3 ? bufs[i] : nullptr;
    hipLaunchKernelGGL(k_diag, dim3(ntasks), dim3(256), 0, c->stream, b, tasks, terms);
    LAUNCHCHK(c);
    return 0;
}

// ================================================== segment dot products
// One work-group per segment: waves stride over rows, lanes over columns.
__global__ void __launch_bounds__(256) k_seg_dots(DBufs bufs, const SegDot* __restrict__ segs,
                                                  double* __restrict__ partial) {
    const SegDot s = segs[blockIdx.x];
    const double* A = bufs.p[s.a_buf] + s.a_off;
    const double* B = bufs.p[s.b_buf] + s.b_off;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    double acc = 0.0;
    for (int r = wave; r < s.rows; r += 4) {
        const double* a = A + (int64_t)r * s.lda;
        const double* b = B + (int64_t)r * s.ldb;
        for (int c = lane; c < s.cols; c += 64) acc += a[c] * b[c];
    }
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o, 64);
    __shared__ double sh[4];
    if (lane == 0) sh[wave] = acc;
    __syncthreads();
    if (threadIdx.x == 0) partial[blockIdx.x] = s.coef * (((sh[0] + sh[1]) + sh[2]) + sh[3]);
}

__global__ void __launch_bounds__(256) k_seg_sum(const double* __restrict__ partial,
                                                 const int32_t* __restrict__ obeg, int nout,
                                                 double* __restrict__ out) {
    const int o = blockIdx.x * blockDim.x + threadIdx.x;
    if (o >= nout) return;
    double s = 0.0;
    for (int t = obeg[o]; t < obeg[o + 1]; ++t) s += partial[t];
    out[o] = s;
}

int seg_dots(Ctx* c, double* const* bufs, const SegDot* segs, int nseg, const int32_t* obeg, int nout,
             double* partial, double* out) {
    if (nout <= 0) return 0;
    DBufs b;
    for (int i = 0; i < kMaxBufs; ++i) b.p[i] = i < 3 ? bufs[i] : nullptr;
    if (nseg > 0) {
        hipLaunchKernelGGL(k_seg_dots, dim3(nseg), dim3(256), 0, c->stream, b, segs, partial);
        LAUNCHCHK(c);
    }
    hipLaunchKernelGGL(k_seg_sum, dim3((nout + 255) / 256), dim3(256), 0, c->stream, partial, obeg, nout, out);
    LAUNCHCHK(c);
    return 0;
}

// ============================================================ FP64 vectors
constexpr int kDotBlocks = 512;

// partial[v * gridDim.x + block] = sum over this block's slice of V_v . w
__global__ void __launch_bounds__(256) k_dots_partial(const double* __restrict__ V, int64_t ldv, int nvec,
                                                      const double* __restrict__ w, int64_t n,
                                                      double* __restrict__ partial) {
    __shared__ double sh[32][8];
    double acc[32];
#pragma unroll
    for (int v = 0; v < 32; ++v) acc[v] = 0.0;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        const double wi = w[i];
#pragma unroll
        for (int v = 0; v < 32; ++v)
            if (v < nvec) acc[v] += V[(int64_t)v * ldv + i] * wi;
    }
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
    for (int v = 0; v < 32; ++v) {
        if (v >= nvec) break;
        double s = acc[v];
        for (int o = 32; o > 0; o >>= 1) s += __shfl_xor(s, o, 64);
        if (lane == 0) sh[v][wave] = s;
    }
    __syncthreads();
    if (threadIdx.x < nvec) {
        double s = 0.0;
        for (int x = 0; x < 4; ++x) s += sh[threadIdx.x][x];
        partial[(int64_t)threadIdx.x * gridDim.x + blockIdx.x] = s;
    }
}

__global__ void __launch_bounds__(256) k_dots_final(const double* __restrict__ partial, int nblk,
                                                    double* __restrict__ out, int ostride) {
    __shared__ double sh[256];
    const int v = blockIdx.x;
    double s = 0.0;
    for (int i = threadIdx.x; i < nblk; i += blockDim.x) s += partial[(int64_t)v * nblk + i];
    sh[threadIdx.x] = s;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
        __syncthreads();
    }
    if (threadIdx.x == 0) out[(int64_t)v * ostride] = sh[0];
}

static int ensure_red(Ctx* c, size_t elems) {
    if (c->red_cap >= elems) return 0;
    if (c->red) hipFree(c->red);
    c->red = nullptr;
    c->red_cap = 0;
    HIPCHK(c, hipMalloc(&c->red, elems * sizeof(double)));
    c->red_cap = elems;
    return 0;
}

int dots(Ctx* c, const double* V, int64_t ldv, int nvec, const double* w, int64_t n, double* out, int ostride) {
    if (nvec <= 0) return 0;
    if (nvec > 32) {
        c->err = "dots: at most 32 vectors";
        return 1;
    }
    int nblk = (int)std::min<int64_t>(kDotBlocks, std::max<int64_t>(1, (n + 255) / 256));
    if (ensure_red(c, (size_t)32 * kDotBlocks)) return 1;
    hipLaunchKernelGGL(k_dots_partial, dim3(nblk), dim3(256), 0, c->stream, V, ldv, nvec, w, n, c->red);
    LAUNCHCHK(c);
    hipLaunchKernelGGL(k_dots_final, dim3(nvec), dim3(256), 0, c->stream, c->red, nblk, out, ostride);
    LAUNCHCHK(c);
    return 0;
}

__global__ void k_combine(const double* __restrict__ V, int64_t ldv, int nvec, const double* __restrict__ coef,
                          double scale, int64_t n, double* __restrict__ out, int accumulate) {
    __shared__ double cf[32];
    if (threadIdx.x < nvec) cf[threadIdx.x] = coef[threadIdx.x] * scale;
    __syncthreads();
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double s = accumulate ? out[i] : 0.0;
        for (int v = 0; v < nvec; ++v) s += cf[v] * V[(int64_t)v * ldv + i];
        out[i] = s;
    }
}
int combine(Ctx* c, const double* V, int64_t ldv, int nvec, const double* coef, double scale, int64_t n,
            double* out, int accumulate) {
    if (n <= 0 || nvec <= 0) return 0;
    hipLaunchKernelGGL(k_combine, dim3(grid_for(n)), dim3(256), 0, c->stream, V, ldv, nvec, coef, scale, n, out,
                       accumulate);
    LAUNCHCHK(c);
    return 0;
}

__global__ void k_residual(const double* __restrict__ hx, const double* __restrict__ x,
                           const double* __restrict__ th, int64_t n, double* __restrict__ r) {
    const double t = *th;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        r[i] = hx[i] - t * x[i];
}
int residual(Ctx* c, const double* hx, const double* x, const double* th, int64_t n, double* r, double* n2) {
    hipLaunchKernelGGL(k_residual, dim3(grid_for(n)), dim3(256), 0, c->stream, hx, x, th, n, r);
    LAUNCHCHK(c);
    return dots(c, r, 0, 1, r, n, n2, 1);
}

__global__ void k_precond(const double* __restrict__ r, const double* __restrict__ d,
                          const double* __restrict__ th, int64_t n, double* __restrict__ t) {
    const double tt = *th;
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
        double den = d[i] - tt;
        if (fabs(den) < 1e-12) den = den < 0.0 ? -1e-12 : 1e-12;
        t[i] = r[i] / den;
    }
}
int precond(Ctx* c, const double* r, const double* d, const double* th, int64_t n, double* t) {
    hipLaunchKernelGGL(k_precond, dim3(grid_for(n)), dim3(256), 0, c->stream, r, d, th, n, t);
    LAUNCHCHK(c);
    return 0;
}

__global__ void k_scale_copy(const double* __restrict__ x, int64_t n, const double* __restrict__ n2,
                             double* __restrict__ y) {
    const double f = 1.0 / sqrt(*n2);
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = x[i] * f;
}
int scale_inv_norm(Ctx* c, double* x, int64_t n, const double* n2) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, c->stream, x, n, n2, x);
    LAUNCHCHK(c);
    return 0;
}
int copy_scaled_inv_norm(Ctx* c, const double* x, int64_t n, const double* n2, double* y) {
    hipLaunchKernelGGL(k_scale_copy, dim3(grid_for(n)), dim3(256), 0, c->stream, x, n, n2, y);
    LAUNCHCHK(c);
    return 0;
}

// Lowest eigenpair of a k x k symmetric matrix (k <= 32): one wave, cyclic
// Jacobi with the round-robin pair schedule (k/2 disjoint rotations per
// round; in round r position i holds index 0 for i = 0, else
// 1 + (i - 1 + r) mod (kk - 1)).  Stops when the off-diagonal norm is below
// 1e-14 of the matrix norm (eigenvalue error ~ its square).
__global__ void __launch_bounds__(64) k_small_eigh(const double* __restrict__ G, int k, int ldg,
                                                   double* __restrict__ theta, double* __restrict__ s) {
    __shared__ double A[32][33];
    __shared__ double Vm[32][33];
    __shared__ double cs[16][2];
    __shared__ int pr[16][2];
    __shared__ double red[64];
    const int t = threadIdx.x;
    const int kk = (k + 1) & ~1;   // even size; a padded index is never rotated
    for (int e = t; e < 32 * 32; e += 64) {
        int i = e >> 5, j = e & 31;
        double v = 0.0;
        if (i < k && j < k) v = i >= j ? G[i * ldg + j] : G[j * ldg + i];
        A[i][j] = v;
        Vm[i][j] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
    for (int sweep = 0; sweep < 30 && kk > 1; ++sweep) {
        double off = 0.0, tot = 0.0;
        for (int e = t; e < k * k; e += 64) {
            int i = e / k, j = e % k;
            double v = A[i][j] * A[i][j];
            tot += v;
            if (i != j) off += v;
        }
        for (int o = 32; o > 0; o >>= 1) {
            off += __shfl_xor(off, o, 64);
            tot += __shfl_xor(tot, o, 64);
        }
        if (off <= 1e-28 * tot || off < 1e-300) break;
        for (int round = 0; round < kk - 1; ++round) {
            if (t < kk / 2) {
                const int i1 = t, i2 = kk - 1 - t;
                int p = i1 == 0 ? 0 : 1 + (i1 - 1 + round) % (kk - 1);
                int q = 1 + (i2 - 1 + round) % (kk - 1);
                if (p > q) {
                    int x = p;
                    p = q;
                    q = x;
                }
                pr[t][0] = p;
                pr[t][1] = q;
                double c = 1.0, sn = 0.0;
                if (q < k) {
                    double apq = A[p][q];
                    if (fabs(apq) > 1e-300) {
                        double th = (A[q][q] - A[p][p]) / (2.0 * apq);
                        double tt = (th >= 0.0 ? 1.0 : -1.0) / (fabs(th) + sqrt(th * th + 1.0));
                        c = 1.0 / sqrt(tt * tt + 1.0);
                        sn = tt * c;
                    }
                }
                cs[t][0] = c;
                cs[t][1] = sn;
            }
            __syncthreads();
            // lane t: pair t % 16, rows (or columns) t / 16 + 4 m
            const int pi = t & 15, g = t >> 4;
            if (pi < kk / 2 && pr[pi][1] < k) {
                const int p = pr[pi][0], q = pr[pi][1];
                const double c = cs[pi][0], sn = cs[pi][1];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int i = g + 4 * m;
                    if (i < k) {
                        const double aip = A[i][p], aiq = A[i][q];
                        A[i][p] = c * aip - sn * aiq;
                        A[i][q] = sn * aip + c * aiq;
                        const double vip = Vm[i][p], viq = Vm[i][q];
                        Vm[i][p] = c * vip - sn * viq;
                        Vm[i][q] = sn * vip + c * viq;
                    }
                }
            }
            __syncthreads();
            if (pi < kk / 2 && pr[pi][1] < k) {
                const int p = pr[pi][0], q = pr[pi][1];
                const double c = cs[pi][0], sn = cs[pi][1];
#pragma unroll
                for (int m = 0; m < 8; ++m) {
                    const int j = g + 4 * m;
                    if (j < k) {
                        const double apj = A[p][j], aqj = A[q][j];
                        A[p][j] = c * apj - sn * aqj;
                        A[q][j] = sn * apj + c * aqj;
                    }
                }
            }
            __syncthreads();
        }
    }
    if (t == 0) {
        int b = 0;
        for (int i = 1; i < k; ++i)
            if (A[i][i] < A[b][b]) b = i;
        red[0] = A[b][b];
        pr[0][0] = b;
    }
    __syncthreads();
    int b = pr[0][0];
    if (t == 0) *theta = red[0];
    if (t < k) s[t] = Vm[t][b];
}
int small_eigh(Ctx* c, const double* G, int k, int ldg, double* theta, double* s) {
    if (k < 1 || k > 32) {
        c->err = "small_eigh: k must be in 1..32";
        return 1;
    }
    hipLaunchKernelGGL(k_small_eigh, dim3(1), dim3(64), 0, c->stream, G, k, ldg, theta, s);
    LAUNCHCHK(c);
    return 0;
}

// ============================================================ conversions
__global__ void k_f64_to_f32(const double* __restrict__ x, float* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (float)x[i];
}
__global__ void k_f64_to_bf16(const double* __restrict__ x, bf16_t* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = f2bf((float)x[i]);
}
__global__ void k_f32_to_f64(const float* __restrict__ x, double* __restrict__ y, int64_t n) {
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
        y[i] = (double)x[i];
}
int convert(Ctx* c, int fp, const void* src, int tp, void* dst, int64_t n) {
    if (n <= 0) return 0;
    dim3 g(grid_for(n)), b(256);
    if (fp == P_F64 && tp == P_F32)
        hipLaunchKernelGGL(k_f64_to_f32, g, b, 0, c->stream, (const double*)src, (float*)dst, n);
    else if (fp == P_F64 && tp == P_BF16)
        hipLaunchKernelGGL(k_f64_to_bf16, g, b, 0, c->stream, (const double*)src, (bf16_t*)dst, n);
    else if (fp == P_F32 && tp == P_F64)
        hipLaunchKernelGGL(k_f32_to_f64, g, b, 0, c->stream, (const float*)src, (double*)dst, n);
    else {
        c->err = "unsupported conversion";
        return 1;
    }
    LAUNCHCHK(c);
    return 0;
}

// ================================================ dense symmetric eigen
int syevd(Ctx* c, int n, double* A, double* w) {
    if (n <= 0) return 0;
    if (c->syev_cap < (size_t)n) {
        if (c->syev_e) hipFree(c->syev_e);
        c->syev_e = nullptr;
        c->syev_cap = 0;
        HIPCHK(c, hipMalloc(&c->syev_e, (size_t)n * sizeof(double)));
        c->syev_cap = n;
    }
    rocblas_status st = rocsolver_dsyevd(c->blas, rocblas_evect_original, rocblas_fill_upper, n, A, n, w,
                                         c->syev_e, c->info);
    if (st != rocblas_status_success) {
        c->err = std::string("rocsolver_dsyevd failed: ") + rocblas_status_to_string(st);
        return 1;
    }
    return 0;
}

int syevd_batched(Ctx* c, int P, int count, double* A, double* w) {
    if (count <= 0 || P <= 0) return 0;
    size_t need = (size_t)P * count;
    if (c->syev_cap < need) {
        if (c->syev_e) hipFree(c->syev_e);
        c->syev_e = nullptr;
        c->syev_cap = 0;
        HIPCHK(c, hipMalloc(&c->syev_e, need * sizeof(double)));
        c->syev_cap = need;
    }
    if (c->info_cap < (size_t)count) {
        if (c->info) hipFree(c->info);
        c->info = nullptr;
        c->info_cap = 0;
        HIPCHK(c, hipMalloc(&c->info, (size_t)count * sizeof(int)));
        c->info_cap = count;
    }
    rocblas_status st = rocsolver_dsyevd_strided_batched(c->blas, rocblas_evect_original, rocblas_fill_upper, P, A,
                                                         P, (rocblas_stride)P * P, w, P, c->syev_e, P, c->info,
                                                         count);
    if (st != rocblas_status_success) {
        c->err = std::string("rocsolver_dsyevd_strided_batched failed: ") + rocblas_status_to_string(st);
        return 1;
    }
    return 0;
}

// Several size buckets at once.  The rocSOLVER divide-and-conquer solver is a
// long chain of small launches per bucket, so the buckets run concurrently on
// side streams (longest chain first onto the least-loaded stream), each after
// all earlier work of the context stream; the context stream then waits for
// all of them.
int syevd_buckets(Ctx* c, int nb, const int* P, const int* count, double* A, const int64_t* aoff, double* w,
                  const int64_t* woff) {
    if (nb <= 0) return 0;
    if (!c->side_ready) {
        for (int i = 0; i < kSide; ++i) {
            HIPCHK(c, hipStreamCreateWithFlags(&c->side[i], hipStreamNonBlocking));
            if (rocblas_create_handle(&c->side_blas[i]) != rocblas_status_success) {
                c->err = "rocblas_create_handle failed";
                return 1;
            }
            rocblas_set_stream(c->side_blas[i], c->side[i]);
            HIPCHK(c, hipEventCreateWithFlags(&c->side_ev[i], hipEventDisableTiming));
        }
        HIPCHK(c, hipEventCreateWithFlags(&c->fork_ev, hipEventDisableTiming));
        c->side_ready = true;
    }
    // longest chains first onto the least-loaded side stream
    std::vector<int> ord(nb), sid(nb);
    for (int j = 0; j < nb; ++j) ord[j] = j;
    std::sort(ord.begin(), ord.end(), [&](int a, int b) { return P[a] > P[b]; });
    int64_t load[kSide] = {0, 0, 0, 0};
    size_t need_e[kSide] = {0, 0, 0, 0}, need_i[kSide] = {0, 0, 0, 0};
    for (int j : ord) {
        if (count[j] <= 0 || P[j] <= 0) {
            sid[j] = -1;
            continue;
        }
        int best = 0;
        for (int i = 1; i < kSide; ++i)
            if (load[i] < load[best]) best = i;
        sid[j] = best;
        load[best] += P[j];
        need_e[best] = std::max(need_e[best], (size_t)P[j] * count[j]);
        need_i[best] = std::max(need_i[best], (size_t)count[j]);
    }
    for (int i = 0; i < kSide; ++i) {
        if (c->side_ecap[i] < need_e[i]) {
            if (c->side_e[i]) HIPCHK(c, hipFree(c->side_e[i]));
            c->side_e[i] = nullptr;
            c->side_ecap[i] = 0;
            HIPCHK(c, hipMalloc(&c->side_e[i], need_e[i] * sizeof(double)));
            c->side_ecap[i] = need_e[i];
        }
        if (c->side_icap[i] < need_i[i]) {
            if (c->side_info[i]) HIPCHK(c, hipFree(c->side_info[i]));
            c->side_info[i] = nullptr;
            c->side_icap[i] = 0;
            HIPCHK(c, hipMalloc(&c->side_info[i], need_i[i] * sizeof(int)));
            c->side_icap[i] = need_i[i];
        }
    }
    HIPCHK(c, hipEventRecord(c->fork_ev, c->stream));
    for (int i = 0; i < kSide; ++i)
        if (load[i]) HIPCHK(c, hipStreamWaitEvent(c->side[i], c->fork_ev, 0));
    for (int j : ord) {
        const int i = sid[j];
        if (i < 0) continue;
        rocblas_status st = rocsolver_dsyevd_strided_batched(
            c->side_blas[i], rocblas_evect_original, rocblas_fill_upper, P[j], A + aoff[j], P[j],
            (rocblas_stride)P[j] * P[j], w + woff[j], P[j], c->side_e[i], P[j], c->side_info[i], count[j]);
        if (st != rocblas_status_success) {
            c->err = std::string("rocsolver_dsyevd_strided_batched failed: ") + rocblas_status_to_string(st);
            return 1;
        }
    }
    for (int i = 0; i < kSide; ++i)
        if (load[i]) {
            HIPCHK(c, hipEventRecord(c->side_ev[i], c->side[i]));
            HIPCHK(c, hipStreamWaitEvent(c->stream, c->side_ev[i], 0));
        }
    return 0;
}

__global__ void k_pad_init(double* __restrict__ base, int P, const int32_t* __restrict__ nn) {
    const int s = blockIdx.y;
    const int n = nn[s];
    double* A = base + (int64_t)s * P * P;
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < (int64_t)P * P;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int r = (int)(e / P), q = (int)(e % P);
        if (r < n && q < n) continue;
        A[e] = (r == q) ? -1.0 : 0.0;
    }
}
int pad_init(Ctx* c, double* base, int P, int count, const int32_t* d_n) {
    if (count <= 0) return 0;
    unsigned gx = grid_for((int64_t)P * P, 256, 256);
    hipLaunchKernelGGL(k_pad_init, dim3(gx, count), dim3(256), 0, c->stream, base, P, d_n);
    LAUNCHCHK(c);
    return 0;
}

// one block per kept column: sign so that the first largest-|.| entry is positive
__global__ void __launch_bounds__(256) k_gather_evecs(const double* __restrict__ E, int n, int stride,
                                                      const int32_t* __restrict__ idx, int k,
                                                      double* __restrict__ U) {
    __shared__ double bv[256];
    __shared__ int bi[256];
    const int col = blockIdx.x;
    const double* e = E + (int64_t)idx[col] * stride;
    double best = -1.0;
    int besti = 0x7fffffff;
    for (int r = threadIdx.x; r < n; r += blockDim.x) {
        double a = fabs(e[r]);
        if (a > best || (a == best && r < besti)) {
            best = a;
            besti = r;
        }
    }
    bv[threadIdx.x] = best;
    bi[threadIdx.x] = besti;
    __syncthreads();
    for (int o = 128; o > 0; o >>= 1) {
        if (threadIdx.x < o) {
            double a = bv[threadIdx.x + o];
            int ai = bi[threadIdx.x + o];
            if (a > bv[threadIdx.x] || (a == bv[threadIdx.x] && ai < bi[threadIdx.x])) {
                bv[threadIdx.x] = a;
                bi[threadIdx.x] = ai;
            }
        }
        __syncthreads();
    }
    const double sg = e[bi[0]] < 0.0 ? -1.0 : 1.0;
    for (int r = threadIdx.x; r < n; r += blockDim.x) U[(int64_t)r * k + col] = sg * e[r];
}
int gather_evecs(Ctx* c, const double* E, int n, int stride, const int32_t* idx, int k, double* U) {
    if (k <= 0) return 0;
    hipLaunchKernelGGL(k_gather_evecs, dim3(k), dim3(256), 0, c->stream, E, n, stride, idx, k, U);
    LAUNCHCHK(c);
    return 0;
}

}  // namespace dmrgdev
