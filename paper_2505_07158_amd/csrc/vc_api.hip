// vc_api.hip -- the C ABI of libvcipher (include/vcipher.h).
//
// Host side of the path: argument validation, per-stream sequence checks,
// descriptor packing (one pinned staging buffer per call, copied to the
// device on the caller's stream), scratch planning (frames are processed in
// spans whose IR, D and B fit the context's scratch), and the launch
// sequence:
//   encrypt: sha256_subframes (all frames) -> per part: lhcs_chain ->
//            lhcs_keygen -> confuse_xor_enc (one launch per frame shape)
//   decrypt: per part: lhcs_chain -> lhcs_keygen -> confuse_xor_dec
// The chain is the serial spine of a stream (frame t+1 starts from the end
// of frame t), while the keygen and confusion of a frame need only that
// frame's IR.  So:
//  - every chain launch of the context runs on one context-owned chain
//    stream, in call order, after an event recorded on the caller's stream
//    at call entry (the call's inputs are ready);
//  - the scratch is divided into slots; each span of frames whose IR, D and
//    B fit a slot takes the next slot, and its first chain waits until the
//    slot's previous user has finished with it;
//  - each span is cut into parts in call order; keygen and confusion of
//    part k run on side stream k mod s, forked after the chain of part k,
//    so keygen k overlaps the chain of part k+1;
//  - the caller's stream waits for the side streams before the call ends,
//    so the call is stream-ordered as a whole.
// A caller that issues consecutive calls on different streams therefore
// lets the chain of call k+1 start while call k's keygen and confusion run.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <map>
#include <mutex>
#include <new>
#include <tuple>
#include <vector>

#include "../../include/vcipher.h"
#include "vc_internal.hpp"

using namespace vc;

// The allocation-free entry point's device buffer: one per GPU the library
// runs on, held until the process ends.  Host code must never pass this
// name to a kernel or a copy (in host code it is a stand-in, not a device
// address); it uses the address hipGetSymbolAddress returns for the current
// device (noalloc_base).
static __device__ __align__(256) uint8_t scratch[VC_NOALLOC_SCRATCH_BYTES];

namespace {

constexpr size_t kNoAllocDesc = size_t(1) << 20;                          // descriptors
constexpr size_t kNoAllocData = size_t(VC_NOALLOC_SCRATCH_BYTES) - kNoAllocDesc;  // per-frame buffers

std::mutex g_noalloc_mu;
std::map<int, uint8_t *> g_noalloc_base;  // device -> address of `scratch` on it

// Address of `scratch` on device `dev` (current), resolved once per device.
hipError_t noalloc_base(int dev, uint8_t **out) {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    auto it = g_noalloc_base.find(dev);
    if (it != g_noalloc_base.end()) {
        *out = it->second;
        return hipSuccess;
    }
    void *p = nullptr;
    const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) return e != hipSuccess ? e : hipErrorInvalidSymbol;
    g_noalloc_base[dev] = static_cast<uint8_t *>(p);
    *out = static_cast<uint8_t *>(p);
    return hipSuccess;
}

constexpr size_t kDefaultScratch = size_t(2) << 30;
constexpr uint32_t kMaxN = 1024;
constexpr double kGammaLo = -1.52;
constexpr double kGammaHi = -0.06;
constexpr uint32_t kMaxDim = 65535;
constexpr int kRing = 8;
constexpr int kMaxSide = 8;
constexpr int kMaxSlots = 4;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

bool key_ok(const vc_key &k) {
    return std::isfinite(k.x0) && std::isfinite(k.y0) && std::isfinite(k.z0) && std::isfinite(k.w0) &&
           k.gamma >= kGammaLo && k.gamma <= kGammaHi && k.n >= 1 && k.n <= kMaxN;
}

struct PendingEvent {
    int kernel;
    hipEvent_t a, b;
};

// Restores the caller's current device on scope exit.
struct DeviceGuard {
    int prev = -1;
    bool ok = true;
    explicit DeviceGuard(int dev) {
        if (hipGetDevice(&prev) != hipSuccess) { ok = false; return; }
        if (prev != dev && hipSetDevice(dev) != hipSuccess) ok = false;
    }
    ~DeviceGuard() {
        int cur = -1;
        if (prev >= 0 && hipGetDevice(&cur) == hipSuccess && cur != prev) (void)hipSetDevice(prev);
    }
};

struct Group {  // frames [first, first + count) of the descriptor array share a shape
    uint32_t first, count, w, h;
    int align;  // alignment class every frame of the group meets (launch_shift)
};

struct Chunk {  // one part of a scratch span
    uint32_t desc_begin, desc_end;
    uint32_t run_begin, run_end;
    uint32_t span;
    std::vector<Group> groups;
};

}  // namespace

struct vc_cipher {
    vc_key key{};
    int device = 0;
    uint32_t max_streams = 0;
    double *d_state = nullptr;
    int *d_flags = nullptr;
    std::vector<uint64_t> next_seq;
    uint8_t *d_scratch = nullptr;
    size_t scratch_bytes = 0;
    uint32_t lds_limit = 65536;
    // descriptor staging ring
    uint8_t *h_stage[kRing] = {};
    uint8_t *d_stage[kRing] = {};
    size_t stage_cap[kRing] = {};
    hipEvent_t stage_ev[kRing] = {};
    bool stage_live[kRing] = {};
    int ring = 0;
    // tuning
    uint32_t strip = 0, threads = 0;
    // autotuned (strip, threads) per (w, h, decrypt, passes); used when no
    // fixed tuning is set
    std::map<std::tuple<uint32_t, uint32_t, int, int>, std::pair<uint32_t, uint32_t>> tuned;
    int xcd_map = 1;
    int passes = 2;  // confusion: 2 = row pass + column pass, 1 = single fused pass
    // overlap of the chain with keygen + confusion (streams at default
    // priority, created on first use so that idle contexts hold none)
    uint32_t parts = 3;
    uint32_t nside = 3;
    uint32_t side_base = 0;  // side stream of the next call's first part (rotates across calls)
    uint32_t nslots = 2;
    uint32_t slot_next = 0;
    hipStream_t chain_stream = nullptr;
    hipEvent_t in_ev = nullptr;
    hipStream_t side[kMaxSide] = {};
    hipEvent_t fork_ev[kMaxSide] = {};
    hipEvent_t join_ev[kMaxSide] = {};
    // per scratch slot: events recorded on the worker streams that last used
    // it (index k = side stream k, or the chain stream when there is none)
    hipEvent_t slot_ev[kMaxSlots][kMaxSide] = {};
    bool slot_live[kMaxSlots][kMaxSide] = {};
    // profiling
    bool profile = false;
    std::vector<PendingEvent> pending;
    std::vector<hipEvent_t> spare;
    double acc_ms[K_COUNT] = {};
    uint64_t acc_n[K_COUNT] = {};
    // allocation-free calls (encrypt_frames_noalloc): the device array
    // `scratch` on this context's GPU, a pinned staging buffer for their
    // descriptors, and events that order them with the context's other calls
    uint8_t *na_base = nullptr;
    uint8_t *na_host = nullptr;
    hipEvent_t na_stage_ev = nullptr;  // behind the last no-alloc descriptor copy
    bool na_stage_live = false;
    hipEvent_t na_wait_ev = nullptr;   // the chain stream's work before a no-alloc call
    hipEvent_t na_done_ev = nullptr;   // end of the last no-alloc call's chain work
    bool na_pending = false;           // the chain stream has not waited for na_done_ev yet
    bool in_noalloc = false;           // set while a no-alloc call runs (no profiling events)
    std::mutex mu;
};

namespace vc {
// True when the first and the last byte of [p, p + bytes) lie in memory
// the kernels can address as it is: device or managed memory, or pinned
// host memory mapped at the same address (hipHostMalloc).  Pageable host
// memory is not (no XNACK), and a kernel touching it faults, so buffers the
// kernels access in place are checked before anything is enqueued.  (A
// range whose two ends lie in different allocations with unmapped memory
// between them is not detected: buffers are expected to be one
// allocation.)
bool reachable(const void *p, size_t bytes) {
    if (!p || bytes == 0) return false;
    const uint8_t *b = static_cast<const uint8_t *>(p);
    for (const uint8_t *q : {b, b + (bytes - 1)}) {
        hipPointerAttribute_t at{};
        if (hipPointerGetAttributes(&at, q) != hipSuccess) {
            (void)hipGetLastError();  // leave no error behind for the next launch check
            return false;
        }
        const bool ok = at.type == hipMemoryTypeDevice || at.type == hipMemoryTypeManaged ||
                        at.type == hipMemoryTypeUnified ||
                        (at.type == hipMemoryTypeHost && at.devicePointer == static_cast<const void *>(q));
        if (!ok) return false;
    }
    return true;
}

}  // namespace vc

namespace {
struct CallArgs;
}
static int locked_call(vc_cipher *ctx, const CallArgs &a);

namespace {

int map_err(hipError_t e) {
    if (e == hipSuccess) return VC_OK;
    if (e == hipErrorOutOfMemory) return VC_ENOMEM;
    return VC_EDEVICE;
}

hipEvent_t take_event(vc_cipher *ctx) {
    if (!ctx->spare.empty()) {
        hipEvent_t e = ctx->spare.back();
        ctx->spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

// Launch wrapper: records a pair of events around the launch when profiling.
template <typename F>
hipError_t timed(vc_cipher *ctx, int kernel, hipStream_t s, F &&launch) {
    if (!ctx->profile || ctx->in_noalloc) return launch();
    hipEvent_t a = take_event(ctx), b = take_event(ctx);
    if (!a || !b) return hipErrorOutOfMemory;
    hipError_t e = hipEventRecord(a, s);
    if (e != hipSuccess) return e;
    e = launch();
    if (e != hipSuccess) return e;
    e = hipEventRecord(b, s);
    if (e != hipSuccess) return e;
    ctx->pending.push_back({kernel, a, b});
    return hipSuccess;
}

hipError_t drain_profile(vc_cipher *ctx) {
    for (auto &p : ctx->pending) {
        hipError_t e = hipEventSynchronize(p.b);
        if (e != hipSuccess) return e;
        float ms = 0.f;
        e = hipEventElapsedTime(&ms, p.a, p.b);
        if (e != hipSuccess) return e;
        ctx->acc_ms[p.kernel] += ms;
        ctx->acc_n[p.kernel] += 1;
        ctx->spare.push_back(p.a);
        ctx->spare.push_back(p.b);
    }
    ctx->pending.clear();
    return hipSuccess;
}

// Pinned host + device staging for one call's descriptors.  A slot is
// reused only after the event recorded behind the last kernel that read it.
int stage_acquire(vc_cipher *ctx, size_t bytes, int *slot_out) {
    const int slot = ctx->ring;
    ctx->ring = (ctx->ring + 1) % kRing;
    if (ctx->stage_live[slot]) {
        if (hipEventSynchronize(ctx->stage_ev[slot]) != hipSuccess) return VC_EDEVICE;
        ctx->stage_live[slot] = false;
    }
    if (ctx->stage_cap[slot] < bytes) {
        if (ctx->h_stage[slot]) (void)hipHostFree(ctx->h_stage[slot]);
        if (ctx->d_stage[slot]) (void)hipFree(ctx->d_stage[slot]);
        ctx->h_stage[slot] = nullptr;
        ctx->d_stage[slot] = nullptr;
        ctx->stage_cap[slot] = 0;
        const size_t cap = std::max(align_up(bytes, 4096), size_t(65536));
        if (hipHostMalloc(reinterpret_cast<void **>(&ctx->h_stage[slot]), cap, hipHostMallocDefault) !=
            hipSuccess)
            return VC_ENOMEM;
        if (hipMalloc(reinterpret_cast<void **>(&ctx->d_stage[slot]), cap) != hipSuccess) return VC_ENOMEM;
        ctx->stage_cap[slot] = cap;
    }
    *slot_out = slot;
    return VC_OK;
}

uint64_t frame_bytes(const vc_shape &s) { return 3ull * s.w * s.h; }

// Scratch of one frame: B, D and IR for the key schedule (keysched), plus
// the intermediate image of the two-pass confusion (two_pass).
uint64_t scratch_need(const vc_shape &s, uint32_t n, bool keysched, bool two_pass) {
    const uint64_t L = frame_bytes(s);
    const uint64_t ND = 3ull * s.h + 3ull * s.w;
    uint64_t b = 0;
    if (keysched) b += align_up(L, 256) + align_up(2 * ND, 256) + align_up(64ull * n, 256);
    if (two_pass) b += align_up(L, 256);
    return b;
}

bool overlaps(const uint8_t *a, uint64_t la, const uint8_t *b, uint64_t lb) {
    return a < b + lb && b < a + la;
}

int check_shape(const vc_cipher *ctx, const vc_shape &s, int decrypt, bool uses_n) {
    if (s.c != 3 || s.w < 1 || s.h < 1 || s.w > kMaxDim || s.h > kMaxDim) return VC_EINVAL;
    if (uses_n && ctx->key.n > frame_bytes(s)) return VC_EINVAL;
    // both directions must fit, so that what is encrypted can be decrypted
    // under the same settings
    (void)decrypt;
    const bool fits = ctx->passes == 2 ? shift_max_strip(s.h, ctx->lds_limit) != 0
                                       : confuse_max_strip(0, s.h, ctx->lds_limit) != 0 &&
                                             confuse_max_strip(1, s.h, ctx->lds_limit) != 0;
    if (!fits) return VC_EINVAL;
    return VC_OK;
}

uint32_t pick_strip(const vc_cipher *ctx, int decrypt, uint32_t w, uint32_t h) {
    const uint32_t wcap = std::max<uint32_t>(4, (w + 3) / 4 * 4);
    if (ctx->passes == 2) {
        // strips of bytes: a strip wider than the row is never needed
        const uint32_t bcap = std::max<uint32_t>(4, 1u << (32 - __builtin_clz(std::max<uint32_t>(3 * w, 2) - 1)));
        if (ctx->strip && ctx->strip <= bcap && shift_col_lds_bytes(h, ctx->strip) <= ctx->lds_limit)
            return ctx->strip;
        // the widest strip (up to one 128-byte line) that leaves room for two
        // column-pass workgroups per CU, else the widest that fits: measured
        // on MI355X, the column pass then shares CUs best with the
        // latency-bound SHA-256 and keystream waves of a pipelined stream
        uint32_t half = 0, fits = 0;
        for (uint32_t sb = 4; sb <= 128 && sb <= bcap; sb *= 2) {
            if (shift_col_lds_bytes(h, sb) <= ctx->lds_limit / 2) half = sb;
            if (shift_col_lds_bytes(h, sb) <= ctx->lds_limit) fits = sb;
        }
        return half ? half : fits;
    }
    if (ctx->strip && ctx->strip <= 64) {
        if (ctx->strip <= wcap && confuse_lds_bytes(decrypt, h, ctx->strip) <= ctx->lds_limit)
            return ctx->strip;
    }
    // Measured on MI355X (1080p, 300 frames): encryption is fastest with
    // the widest strip that fits the LDS (one workgroup per CU), decryption
    // with the widest strip that leaves room for two workgroups per CU.
    uint32_t half = 0, fits = 0;
    for (uint32_t wt = 4; wt <= 64 && wt <= wcap; wt *= 2) {
        if (confuse_lds_bytes(decrypt, h, wt) <= ctx->lds_limit / 2) half = wt;
        if (confuse_lds_bytes(decrypt, h, wt) <= ctx->lds_limit) fits = wt;
    }
    if (decrypt) return half ? half : fits;
    return fits;
}

// The confusion tiling of a shape: the context's fixed tiling, else the
// autotuned one, else the default strip.  The strip-major layout of the
// intermediate image uses the same strip width.
ConfuseTuning choose_tiling(const vc_cipher *ctx, int decrypt, uint32_t w, uint32_t h) {
    ConfuseTuning t;
    t.strip = pick_strip(ctx, decrypt, w, h);
    t.threads = ctx->threads ? ctx->threads : 1024;
    t.xcd_map = ctx->xcd_map;
    if (!ctx->strip && !ctx->threads) {
        auto it = ctx->tuned.find(std::make_tuple(w, h, decrypt, ctx->passes));
        if (it != ctx->tuned.end()) {
            t.strip = it->second.first;
            t.threads = it->second.second;
        }
    }
    return t;
}


enum class Op { Encrypt, EncryptHashed, Decrypt, Hash, DebugConfuse, DebugKeysched, DebugKeygen };

struct CallArgs {
    Op op;
    size_t count;
    const uint8_t *const *in;
    const vc_shape *shapes;
    const uint8_t *hashes;       // H in (decrypt, keysched)
    uint8_t *hashes_out;         // H out (encrypt, hash)
    uint8_t *const *hash_ptrs;   // per-frame H (32 bytes each) in place of hashes / hashes_out
    uint8_t *const *out;
    const uint16_t *const *dbgD;  // debug confuse inputs
    const uint8_t *const *dbgB;
    double *const *kIR;           // debug keysched outputs (debug keygen: input)
    uint16_t *const *kD;
    uint8_t *const *kB;
    int decrypt;                  // for DebugConfuse
    bool noalloc;                 // encrypt_frames_noalloc: buffers in `scratch`, everything on `stream`
    hipStream_t stream;
};

hipError_t ensure_streams(vc_cipher *ctx) {
    hipError_t e = hipSuccess;
    if (!ctx->chain_stream) {
        e = hipEventCreateWithFlags(&ctx->in_ev, hipEventDisableTiming);
        for (int k = 0; k < kMaxSide && e == hipSuccess; ++k) {
            e = hipEventCreateWithFlags(&ctx->fork_ev[k], hipEventDisableTiming);
            if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->join_ev[k], hipEventDisableTiming);
            for (int q = 0; q < kMaxSlots && e == hipSuccess; ++q)
                e = hipEventCreateWithFlags(&ctx->slot_ev[q][k], hipEventDisableTiming);
        }
        if (e == hipSuccess) e = hipStreamCreateWithFlags(&ctx->chain_stream, hipStreamNonBlocking);
    }
    for (uint32_t k = 0; k < ctx->nside && e == hipSuccess; ++k)
        if (!ctx->side[k]) e = hipStreamCreateWithFlags(&ctx->side[k], hipStreamNonBlocking);
    return e;
}

size_t slot_bytes(const vc_cipher *ctx) { return ctx->scratch_bytes / ctx->nslots / 256 * 256; }

// A call's work, planned on the host: spans of consecutive frames whose
// scratch fits `cap` bytes (span j's buffers start at span_base(j)), each
// cut into up to `nparts` parts in call order; per part the frame
// descriptors grouped by shape and alignment class, and the per-stream runs
// of chain records.
struct Plan {
    std::vector<FrameDesc> desc;
    std::vector<StreamRun> runs;
    std::vector<ChainRec> order;
    std::vector<Chunk> chunks;
    uint32_t nspans = 0;
};

template <typename SpanBase>
void build_plan(const vc_cipher *ctx, const CallArgs &a, bool keysched_scratch, bool two_pass, bool uses_chain,
                bool uses_scratch, int dec_kernel, uint64_t cap, size_t nparts, SpanBase span_base, Plan &P) {
    const size_t count = a.count;
    const uint32_t n = ctx->key.n;
    struct Part {
        size_t b, e;
        uint32_t span;
    };
    std::vector<Part> parts;  // [b, e) in call order
    {
        std::vector<std::pair<size_t, size_t>> spans;
        size_t b = 0;
        uint64_t used = 0;
        for (size_t f = 0; f < count; ++f) {
            const uint64_t need = uses_scratch ? scratch_need(a.shapes[f], n, keysched_scratch, two_pass) : 0;
            if (f > b && used + need > cap) {
                spans.push_back({b, f});
                b = f;
                used = 0;
            }
            used += need;
        }
        spans.push_back({b, count});
        for (size_t si = 0; si < spans.size(); ++si) {
            const size_t sb = spans[si].first, len = spans[si].second - sb;
            const size_t np = std::max<size_t>(1, std::min<size_t>(nparts, len));
            for (size_t k = 0; k < np; ++k)
                parts.push_back({sb + len * k / np, sb + len * (k + 1) / np, static_cast<uint32_t>(si)});
        }
    }

    // descriptors, runs and chain records
    std::vector<FrameDesc> &desc = P.desc;
    std::vector<StreamRun> &runs = P.runs;
    std::vector<ChainRec> &order = P.order;
    std::vector<Chunk> &chunks = P.chunks;
    desc.assign(count, FrameDesc{});
    std::vector<uint32_t> desc_of(count);
    P.nspans = parts.empty() ? 0 : parts.back().span + 1;
    uint8_t *sbase = nullptr;
    uint64_t off = 0;
    for (size_t pi = 0; pi < parts.size(); ++pi) {
        const Part &pt = parts[pi];
        const std::pair<size_t, size_t> sp{pt.b, pt.e};
        if (pi == 0 || parts[pi - 1].span != pt.span) {
            sbase = span_base(pt.span);
            off = 0;
        }
        Chunk ch;
        ch.span = pt.span;
        ch.desc_begin = static_cast<uint32_t>(sp.first);
        ch.desc_end = static_cast<uint32_t>(sp.second);
        // shape groups: stable order by (w, h, alignment class)
        std::vector<size_t> idx;
        for (size_t f = sp.first; f < sp.second; ++f) idx.push_back(f);
        // alignment class (launch_shift): 2 = rows and pointers 16-byte
        // aligned, 1 = 4-byte aligned, 0 = neither
        auto align_of = [&](size_t f) {
            const vc_shape &s = a.shapes[f];
            uintptr_t p = reinterpret_cast<uintptr_t>(a.in ? a.in[f] : nullptr) |
                          reinterpret_cast<uintptr_t>(a.out ? a.out[f] : nullptr);
            if (a.op == Op::DebugConfuse) p |= reinterpret_cast<uintptr_t>(a.dbgB[f]);
            if (s.w % 4 || (p & 3)) return 0;
            return (s.w % 16 == 0 && (p & 15) == 0) ? 2 : 1;
        };
        std::stable_sort(idx.begin(), idx.end(), [&](size_t x, size_t y) {
            const vc_shape &p = a.shapes[x], &q = a.shapes[y];
            return std::make_tuple(p.w, p.h, -align_of(x)) < std::make_tuple(q.w, q.h, -align_of(y));
        });
        for (size_t k = 0; k < idx.size(); ++k) {
            const size_t f = idx[k];
            const uint32_t di = static_cast<uint32_t>(sp.first + k);
            desc_of[f] = di;
            const vc_shape &s = a.shapes[f];
            FrameDesc &d = desc[di];
            d.in = a.in ? a.in[f] : nullptr;
            d.out = a.out ? a.out[f] : nullptr;
            d.w = s.w;
            d.h = s.h;
            d.L = frame_bytes(s);
            d.hash = a.hash_ptrs    ? a.hash_ptrs[f]
                     : a.hashes_out ? a.hashes_out + 32 * f
                                    : const_cast<uint8_t *>(a.hashes ? a.hashes + 32 * f : nullptr);
            d.IR = nullptr;
            d.D = nullptr;
            d.B = nullptr;
            d.X = nullptr;
            d.xstrip = 0;
            d.pad = 0;
            if (two_pass) {
                d.X = sbase + off;
                off += align_up(d.L, 256);
                // strip-major intermediate in the column pass's strips
                d.xstrip = shift_xstrip(s.w, choose_tiling(ctx, dec_kernel, s.w, s.h).strip, align_of(f),
                                        ctx->lds_limit);
            }
            if (keysched_scratch) {
                const uint64_t ND = 3ull * s.h + 3ull * s.w;
                d.B = sbase + off;
                off += align_up(d.L, 256);
                d.D = reinterpret_cast<uint16_t *>(sbase + off);
                off += align_up(2 * ND, 256);
                d.IR = reinterpret_cast<double *>(sbase + off);
                off += align_up(64ull * n, 256);
            } else if (a.op == Op::DebugConfuse) {
                d.D = const_cast<uint16_t *>(a.dbgD[f]);
                d.B = const_cast<uint8_t *>(a.dbgB[f]);
            } else if (a.op == Op::DebugKeysched || a.op == Op::DebugKeygen) {
                d.IR = a.kIR[f];
                d.D = a.kD[f];
                d.B = a.kB[f];
            }
            const int al = align_of(f);
            if (!ch.groups.empty()) {
                Group &g = ch.groups.back();
                if (g.w == s.w && g.h == s.h && g.align == al) {
                    g.count++;
                    continue;
                }
            }
            ch.groups.push_back({di, 1, s.w, s.h, al});
        }
        // stream runs in call (= sequence) order
        ch.run_begin = static_cast<uint32_t>(runs.size());
        if (uses_chain) {
            std::map<uint32_t, std::vector<uint32_t>> per_stream;
            std::vector<uint32_t> stream_order;
            for (size_t f = sp.first; f < sp.second; ++f) {
                auto &v = per_stream[a.shapes[f].stream];
                if (v.empty()) stream_order.push_back(a.shapes[f].stream);
                v.push_back(desc_of[f]);
            }
            for (uint32_t st : stream_order) {
                auto &v = per_stream[st];
                runs.push_back({st, static_cast<uint32_t>(order.size()), static_cast<uint32_t>(v.size()), 0});
                for (uint32_t di : v) order.push_back({desc[di].hash, desc[di].IR});
            }
        }
        ch.run_end = static_cast<uint32_t>(runs.size());
        chunks.push_back(std::move(ch));
    }

}

int run_call(vc_cipher *ctx, const CallArgs &a) {
    const bool encrypting = a.op == Op::Encrypt || a.op == Op::EncryptHashed;
    const bool uses_chain = encrypting || a.op == Op::Decrypt || a.op == Op::DebugKeysched;
    const bool keysched_scratch = encrypting || a.op == Op::Decrypt;
    const bool two_pass =
        ctx->passes == 2 && a.op != Op::Hash && a.op != Op::DebugKeysched && a.op != Op::DebugKeygen;
    const bool uses_scratch = keysched_scratch || two_pass;
    const int dec_kernel = (a.op == Op::Decrypt) || (a.op == Op::DebugConfuse && a.decrypt);
    const uint32_t n = ctx->key.n;
    const size_t count = a.count;

    // ---- validation (nothing enqueued yet) ----
    std::map<uint32_t, uint64_t> seq_next;
    for (size_t f = 0; f < count; ++f) {
        const vc_shape &s = a.shapes[f];
        int rc = check_shape(ctx, s, dec_kernel, a.op != Op::DebugConfuse);
        if (rc) return rc;
        const uint64_t L = frame_bytes(s);
        if (a.op != Op::DebugKeysched && a.op != Op::DebugKeygen && !a.in[f]) return VC_EINVAL;
        if ((encrypting || a.op == Op::Decrypt || a.op == Op::DebugConfuse) && !a.out[f]) return VC_EINVAL;
        if ((encrypting || a.op == Op::DebugConfuse || a.op == Op::Decrypt) && overlaps(a.in[f], L, a.out[f], L))
            return VC_EINVAL;
        if (a.op == Op::DebugConfuse && (!a.dbgD[f] || !a.dbgB[f])) return VC_EINVAL;
        if ((a.op == Op::DebugKeysched || a.op == Op::DebugKeygen) && (!a.kIR[f] || !a.kD[f] || !a.kB[f]))
            return VC_EINVAL;
        if (uses_scratch && scratch_need(s, n, keysched_scratch, two_pass) > (a.noalloc ? kNoAllocData : slot_bytes(ctx)))
            return VC_ENOMEM;
        if (uses_chain) {
            if (s.stream >= ctx->max_streams) return VC_EINVAL;
            auto it = seq_next.find(s.stream);
            const uint64_t expect = (it == seq_next.end()) ? ctx->next_seq[s.stream] : it->second;
            if (s.seq != expect) return VC_EORDER;
            seq_next[s.stream] = expect + 1;
        }
    }
    // hash buffers are read and written by the kernels in place: device
    // memory or pinned host memory only (pageable memory would fault)
    if (count) {
        if (a.hash_ptrs) {
            for (size_t f = 0; f < count; ++f)
                if (!reachable(a.hash_ptrs[f], 32)) return VC_EINVAL;
        } else {
            const uint8_t *hb = a.hashes_out ? a.hashes_out : a.hashes;
            if (hb && !reachable(hb, 32 * count)) return VC_EINVAL;
        }
    }
    // descriptors of a no-alloc call: frame descriptors, at most one stream
    // run and one chain record per frame, each table 256-byte aligned
    if (a.noalloc && align_up(sizeof(FrameDesc) * count, 256) + align_up(sizeof(StreamRun) * count, 256) +
                             align_up(sizeof(ChainRec) * count, 256) > kNoAllocDesc)
        return VC_EINVAL;
    if (count == 0) return VC_OK;
    if ((uses_chain || uses_scratch) && !a.noalloc) {
        const hipError_t e = ensure_streams(ctx);
        if (e != hipSuccess) return map_err(e);
    }

    // ---- plan spans (consecutive frames whose scratch fits a slot) and parts ----
    const bool overlap = (encrypting || a.op == Op::Decrypt) && ctx->parts > 1 && !a.noalloc;
    const size_t cap = a.noalloc ? kNoAllocData : slot_bytes(ctx);
    Plan P;
    // span j of a call uses scratch slot (slot_next + j) mod nslots; a no-alloc
    // call reuses the data area of `scratch` for every span (one stream)
    build_plan(ctx, a, keysched_scratch, two_pass, uses_chain, uses_scratch, dec_kernel, cap,
               overlap ? ctx->parts : 1,
               [&](uint32_t span) {
                   return a.noalloc ? ctx->na_base + kNoAllocDesc
                                    : ctx->d_scratch + ((ctx->slot_next + span) % ctx->nslots) * cap;
               },
               P);
    const std::vector<FrameDesc> &desc = P.desc;
    const std::vector<StreamRun> &runs = P.runs;
    const std::vector<ChainRec> &order = P.order;
    const std::vector<Chunk> &chunks = P.chunks;
    const uint32_t nspans = P.nspans;
    auto slot_of = [&](uint32_t span) { return (ctx->slot_next + span) % ctx->nslots; };

    // ---- stage and upload ----
    const size_t desc_bytes = align_up(sizeof(FrameDesc) * count, 256);
    const size_t runs_bytes = align_up(sizeof(StreamRun) * std::max<size_t>(runs.size(), 1), 256);
    const size_t order_bytes = align_up(sizeof(ChainRec) * std::max<size_t>(order.size(), 1), 256);
    const size_t total = desc_bytes + runs_bytes + order_bytes;
    int slot = 0;
    uint8_t *hs = nullptr, *ds = nullptr;
    if (a.noalloc) {
        // the pinned buffer from cipher_init, once the previous no-alloc
        // call's copy out of it is done; the descriptors go to the head of
        // `scratch`
        if (ctx->na_stage_live && hipEventSynchronize(ctx->na_stage_ev) != hipSuccess) return VC_EDEVICE;
        ctx->na_stage_live = false;
        hs = ctx->na_host;
        ds = ctx->na_base;
    } else {
        int rc = stage_acquire(ctx, total, &slot);
        if (rc) return rc;
        hs = ctx->h_stage[slot];
        ds = ctx->d_stage[slot];
    }
    std::memcpy(hs, desc.data(), sizeof(FrameDesc) * count);
    if (!runs.empty()) std::memcpy(hs + desc_bytes, runs.data(), sizeof(StreamRun) * runs.size());
    if (!order.empty()) std::memcpy(hs + desc_bytes + runs_bytes, order.data(), sizeof(ChainRec) * order.size());
    const hipStream_t s = a.stream;
    hipError_t e = hipMemcpyAsync(ds, hs, total, hipMemcpyHostToDevice, s);
    if (e != hipSuccess) return map_err(e);
    if (a.noalloc) {
        e = hipEventRecord(ctx->na_stage_ev, s);
        if (e != hipSuccess) return map_err(e);
        ctx->na_stage_live = true;
    }
    const FrameDesc *d_desc = reinterpret_cast<const FrameDesc *>(ds);
    const StreamRun *d_runs = reinterpret_cast<const StreamRun *>(ds + desc_bytes);
    const ChainRec *d_order = reinterpret_cast<const ChainRec *>(ds + desc_bytes + runs_bytes);

    // The sequence numbers advance as soon as work is enqueued: the chain
    // states on the device follow stream order.
    if (uses_chain)
        for (auto &kv : seq_next) ctx->next_seq[kv.first] = kv.second;

    ConfuseTuning tun;
    tun.threads = ctx->threads ? ctx->threads : 1024;
    tun.xcd_map = ctx->xcd_map;

    // Confusion + XOR (or its inverse) of one shape group on stream ws.
    auto confuse_group = [&](const Group &g, hipStream_t ws) {
        tun = choose_tiling(ctx, dec_kernel, g.w, g.h);
        if (!two_pass)
            return timed(ctx, dec_kernel ? K_DEC : K_ENC, ws, [&] {
                return launch_confuse(dec_kernel, d_desc, g.first, g.count, g.w, g.h, g.align >= 1, tun, ws);
            });
        for (int pass = 0; pass < 2; ++pass) {
            const int kid = dec_kernel ? (pass == 0 ? K_COL_DEC : K_ROW_DEC) : (pass == 0 ? K_ROW_ENC : K_COL_ENC);
            const hipError_t pe = timed(ctx, kid, ws, [&] {
                return launch_shift(dec_kernel, pass, d_desc, g.first, g.count, g.w, g.h, g.align, tun,
                                    ctx->lds_limit, ws);
            });
            if (pe != hipSuccess) return pe;
        }
        return hipSuccess;
    };

    // ---- launches ----
    if (a.op == Op::Encrypt || a.op == Op::Hash) {
        e = timed(ctx, K_SHA, s, [&] { return launch_sha256_subframes(d_desc, static_cast<uint32_t>(count), n, s); });
        if (e != hipSuccess) return map_err(e);
    }
    if (a.op == Op::DebugKeygen) {
        e = timed(ctx, K_KEYGEN, s, [&] {
            return launch_lhcs_keygen(d_desc, static_cast<uint32_t>(count), n, ctx->key.gamma, ctx->d_flags, s);
        });
        if (e != hipSuccess) return map_err(e);
    }
    if (uses_chain) {
        // a no-alloc call runs its chain, keygen and confusion on the caller's
        // stream (no stream or event of its own is created)
        hipStream_t cs = a.noalloc ? s : ctx->chain_stream;
        // worker streams for keygen + confusion: the side streams, or the
        // chain stream itself when there are none
        const bool sides = ctx->nside && !a.noalloc;
        const uint32_t nw = sides ? ctx->nside : 1;
        auto wstream = [&](uint32_t k) { return sides ? ctx->side[k] : cs; };
        bool used_call[kMaxSide] = {}, used_span[kMaxSide] = {};
        auto release_span = [&](uint32_t span) {
            hipError_t re = hipSuccess;
            if (a.noalloc) return re;  // `scratch` is not divided into slots
            const uint32_t q = slot_of(span);
            for (uint32_t k = 0; k < nw; ++k) {
                if (!used_span[k]) continue;
                used_span[k] = false;
                const hipError_t x = hipEventRecord(ctx->slot_ev[q][k], wstream(k));
                if (x == hipSuccess) ctx->slot_live[q][k] = true;
                if (re == hipSuccess) re = x;
            }
            return re;
        };
        // Makes the caller's stream wait for every worker stream of the call.
        auto join = [&]() {
            hipError_t je = hipSuccess;
            if (a.noalloc) return je;  // everything ran on the caller's stream
            for (uint32_t k = 0; k < nw; ++k) {
                if (!used_call[k]) continue;
                used_call[k] = false;
                hipError_t x = hipEventRecord(ctx->join_ev[k], wstream(k));
                if (x == hipSuccess) x = hipStreamWaitEvent(s, ctx->join_ev[k], 0);
                if (je == hipSuccess) je = x;
            }
            return je;
        };
        int cur_span = -1;
        auto fail = [&](hipError_t err) {
            if (cur_span >= 0 && uses_scratch) (void)release_span(static_cast<uint32_t>(cur_span));
            (void)join();
            return map_err(err);
        };
        if (a.noalloc) {
            // after the chain work of the context's earlier calls (the chain
            // states are shared)
            if (ctx->chain_stream) {
                e = hipEventRecord(ctx->na_wait_ev, ctx->chain_stream);
                if (e == hipSuccess) e = hipStreamWaitEvent(s, ctx->na_wait_ev, 0);
            }
        } else {
            e = hipEventRecord(ctx->in_ev, s);
            if (e == hipSuccess) e = hipStreamWaitEvent(cs, ctx->in_ev, 0);
            // and after the last no-alloc call's chain work
            if (e == hipSuccess && ctx->na_pending) {
                e = hipStreamWaitEvent(cs, ctx->na_done_ev, 0);
                if (e == hipSuccess) ctx->na_pending = false;
            }
        }
        if (e != hipSuccess) return map_err(e);
        for (size_t ci = 0; ci < chunks.size(); ++ci) {
            const Chunk &ch = chunks[ci];
            if (static_cast<int>(ch.span) != cur_span) {
                if (cur_span >= 0 && uses_scratch) {
                    e = release_span(static_cast<uint32_t>(cur_span));
                    if (e != hipSuccess) return fail(e);
                }
                cur_span = static_cast<int>(ch.span);
                if (uses_scratch && !a.noalloc) {  // wait until the slot's previous user is done with it
                    const uint32_t q = slot_of(ch.span);
                    for (int k = 0; k < kMaxSide; ++k) {
                        if (!ctx->slot_live[q][k]) continue;
                        e = hipStreamWaitEvent(cs, ctx->slot_ev[q][k], 0);
                        if (e != hipSuccess) return fail(e);
                        ctx->slot_live[q][k] = false;
                    }
                }
            }
            e = timed(ctx, K_CHAIN, cs, [&] {
                return launch_lhcs_chain(d_runs + ch.run_begin, d_order, ch.run_end - ch.run_begin, ctx->d_state, n,
                                         ctx->key.gamma, ctx->d_flags, cs);
            });
            if (e != hipSuccess) return fail(e);
            const uint32_t k = static_cast<uint32_t>((ctx->side_base + ci) % nw);
            hipStream_t ws = wstream(k);
            if (ws != cs) {
                e = hipEventRecord(ctx->fork_ev[k], cs);
                if (e == hipSuccess) e = hipStreamWaitEvent(ws, ctx->fork_ev[k], 0);
                if (e != hipSuccess) return fail(e);
            }
            used_call[k] = used_span[k] = true;
            e = timed(ctx, K_KEYGEN, ws, [&] {
                return launch_lhcs_keygen(d_desc + ch.desc_begin, ch.desc_end - ch.desc_begin, n, ctx->key.gamma,
                                          ctx->d_flags, ws);
            });
            if (e != hipSuccess) return fail(e);
            if (a.op != Op::DebugKeysched) {
                for (const Group &g : ch.groups) {
                    e = confuse_group(g, ws);
                    if (e != hipSuccess) return fail(e);
                }
            }
        }
        if (cur_span >= 0 && uses_scratch) {
            e = release_span(static_cast<uint32_t>(cur_span));
            if (e != hipSuccess) return fail(e);
        }
        e = join();
        if (e != hipSuccess) return map_err(e);
        if (a.noalloc) {
            e = hipEventRecord(ctx->na_done_ev, s);
            if (e != hipSuccess) return map_err(e);
            ctx->na_pending = true;
        } else {
            if (uses_scratch) ctx->slot_next = (ctx->slot_next + nspans) % ctx->nslots;
            // the next call starts on the next side stream, so that the keygen and
            // confusion of consecutive one-part calls overlap
            ctx->side_base = static_cast<uint32_t>((ctx->side_base + chunks.size()) % nw);
        }
    } else if (a.op == Op::DebugConfuse) {
        // On the caller's stream; the two-pass intermediate takes scratch
        // slots like any other call.
        int cur_span = -1;
        for (const Chunk &ch : chunks) {
            if (uses_scratch && static_cast<int>(ch.span) != cur_span) {
                if (cur_span >= 0) {
                    const uint32_t q = slot_of(static_cast<uint32_t>(cur_span));
                    e = hipEventRecord(ctx->slot_ev[q][0], s);
                    if (e != hipSuccess) return map_err(e);
                    ctx->slot_live[q][0] = true;
                }
                cur_span = static_cast<int>(ch.span);
                const uint32_t q = slot_of(ch.span);
                for (int k = 0; k < kMaxSide; ++k) {
                    if (!ctx->slot_live[q][k]) continue;
                    e = hipStreamWaitEvent(s, ctx->slot_ev[q][k], 0);
                    if (e != hipSuccess) return map_err(e);
                    ctx->slot_live[q][k] = false;
                }
            }
            for (const Group &g : ch.groups) {
                e = confuse_group(g, s);
                if (e != hipSuccess) return map_err(e);
            }
        }
        if (uses_scratch && cur_span >= 0) {
            const uint32_t q = slot_of(static_cast<uint32_t>(cur_span));
            e = hipEventRecord(ctx->slot_ev[q][0], s);
            if (e != hipSuccess) return map_err(e);
            ctx->slot_live[q][0] = true;
            ctx->slot_next = (ctx->slot_next + nspans) % ctx->nslots;
        }
    }
    if (!a.noalloc) {
        e = hipEventRecord(ctx->stage_ev[slot], s);
        if (e != hipSuccess) return map_err(e);
        ctx->stage_live[slot] = true;
    }
    return VC_OK;
}

}  // namespace

extern "C" {

uint32_t vc_protocol_version(void) { return 1; }

int encrypt_frames_hashed(vc_cipher *ctx, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                          const uint8_t *hashes, uint8_t *const *out, void *stream) {
    if (count && (!frames || !shapes || !hashes || !out)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::EncryptHashed;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    a.hashes = hashes;
    a.out = out;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

const char *vc_strerror(int status) {
    switch (status) {
    case VC_OK: return "ok";
    case VC_EINVAL: return "invalid argument";
    case VC_ENOMEM: return "out of memory (device scratch or allocation)";
    case VC_EDEVICE: return "HIP runtime error";
    case VC_EORDER: return "frame out of sequence for its stream";
    case VC_ENONFINITE: return "LHCS trajectory became non-finite";
    case VC_EBUSY: return "busy";
    default: return "unknown status";
    }
}

const char *vc_kernel_name(int kernel_id) {
    switch (kernel_id) {
    case K_SHA: return "sha256_subframes";
    case K_CHAIN: return "lhcs_chain";
    case K_KEYGEN: return "lhcs_keygen";
    case K_ENC: return "confuse_xor_enc";
    case K_DEC: return "confuse_xor_dec";
    case K_ROW_ENC: return "row_shift_enc";
    case K_COL_ENC: return "col_shift_xor_enc";
    case K_COL_DEC: return "col_shift_xor_dec";
    case K_ROW_DEC: return "row_shift_dec";
    default: return "";
    }
}

int vc_key_from_bytes(const uint8_t key32[32], double gamma, uint32_t n, vc_key *out) {
    if (!key32 || !out) return VC_EINVAL;
    if (!(gamma >= kGammaLo && gamma <= kGammaHi) || n < 1 || n > kMaxN) return VC_EINVAL;
    double v[4];
    for (int k = 0; k < 4; ++k) {
        const uint8_t *q = key32 + 8 * k;
        const uint32_t ip = ((uint32_t(q[0]) << 8) | q[1]) % 32u;
        uint64_t fr = 0;
        for (int b = 2; b < 8; ++b) fr = (fr << 8) | q[b];
        v[k] = static_cast<double>(ip) + static_cast<double>(fr) * (1.0 / 281474976710656.0);
    }
    out->x0 = v[0];
    out->y0 = v[1];
    out->z0 = v[2];
    out->w0 = v[3];
    out->gamma = gamma;
    out->n = n;
    return VC_OK;
}

void cipher_destroy(vc_cipher *ctx) {
    if (!ctx) return;
    {
        DeviceGuard g(ctx->device);
        (void)hipDeviceSynchronize();
        for (auto &p : ctx->pending) {
            (void)hipEventDestroy(p.a);
            (void)hipEventDestroy(p.b);
        }
        for (auto ev : ctx->spare) (void)hipEventDestroy(ev);
        for (int k = 0; k < kRing; ++k) {
            if (ctx->h_stage[k]) (void)hipHostFree(ctx->h_stage[k]);
            if (ctx->d_stage[k]) (void)hipFree(ctx->d_stage[k]);
            if (ctx->stage_ev[k]) (void)hipEventDestroy(ctx->stage_ev[k]);
        }
        for (int k = 0; k < kMaxSide; ++k) {
            if (ctx->side[k]) (void)hipStreamDestroy(ctx->side[k]);
            if (ctx->fork_ev[k]) (void)hipEventDestroy(ctx->fork_ev[k]);
            if (ctx->join_ev[k]) (void)hipEventDestroy(ctx->join_ev[k]);
            for (int q = 0; q < kMaxSlots; ++q)
                if (ctx->slot_ev[q][k]) (void)hipEventDestroy(ctx->slot_ev[q][k]);
        }
        if (ctx->chain_stream) (void)hipStreamDestroy(ctx->chain_stream);
        if (ctx->in_ev) (void)hipEventDestroy(ctx->in_ev);
        if (ctx->na_host) (void)hipHostFree(ctx->na_host);
        if (ctx->na_stage_ev) (void)hipEventDestroy(ctx->na_stage_ev);
        if (ctx->na_wait_ev) (void)hipEventDestroy(ctx->na_wait_ev);
        if (ctx->na_done_ev) (void)hipEventDestroy(ctx->na_done_ev);
        if (ctx->d_scratch) (void)hipFree(ctx->d_scratch);
        if (ctx->d_state) (void)hipFree(ctx->d_state);
        if (ctx->d_flags) (void)hipFree(ctx->d_flags);
    }
    delete ctx;
}

int cipher_init(const vc_key *key, uint32_t max_streams, size_t scratch_bytes, vc_cipher **out) {
    if (out) *out = nullptr;
    if (!key || !out || max_streams == 0 || !key_ok(*key)) return VC_EINVAL;
    vc_cipher *ctx = new (std::nothrow) vc_cipher();
    if (!ctx) return VC_ENOMEM;
    ctx->key = *key;
    ctx->max_streams = max_streams;
    ctx->scratch_bytes = scratch_bytes ? scratch_bytes : kDefaultScratch;
    int rc = VC_OK;
    do {
        if (hipGetDevice(&ctx->device) != hipSuccess) { rc = VC_EDEVICE; break; }
        int lds = 0;
        if (hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, ctx->device) != hipSuccess) {
            rc = VC_EDEVICE;
            break;
        }
        ctx->lds_limit = static_cast<uint32_t>(lds);
        if (confuse_configure(ctx->lds_limit) != hipSuccess || shift_configure(ctx->lds_limit) != hipSuccess) {
            rc = VC_EDEVICE;
            break;
        }
        try {
            ctx->next_seq.assign(max_streams, 0);
        } catch (...) {
            rc = VC_ENOMEM;
            break;
        }
        hipError_t e = hipMalloc(reinterpret_cast<void **>(&ctx->d_state), sizeof(double) * 4 * max_streams);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&ctx->d_flags), 256);
        if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&ctx->d_scratch), ctx->scratch_bytes);
        if (e != hipSuccess) { rc = map_err(e); break; }
        std::vector<double> st(4ull * max_streams);
        for (uint32_t k = 0; k < max_streams; ++k) {
            st[4 * k] = key->x0;
            st[4 * k + 1] = key->y0;
            st[4 * k + 2] = key->z0;
            st[4 * k + 3] = key->w0;
        }
        e = hipMemcpy(ctx->d_state, st.data(), sizeof(double) * st.size(), hipMemcpyHostToDevice);
        if (e == hipSuccess) e = hipMemset(ctx->d_flags, 0, 256);
        for (int k = 0; k < kRing && e == hipSuccess; ++k) e = hipEventCreateWithFlags(&ctx->stage_ev[k], hipEventDisableTiming);
        // what encrypt_frames_noalloc needs, set up here so that it never
        // allocates: the address of `scratch` on this device, a pinned
        // staging buffer for its descriptors and its ordering events
        if (e == hipSuccess) e = noalloc_base(ctx->device, &ctx->na_base);
        if (e == hipSuccess)
            e = hipHostMalloc(reinterpret_cast<void **>(&ctx->na_host), kNoAllocDesc, hipHostMallocDefault);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->na_stage_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->na_wait_ev, hipEventDisableTiming);
        if (e == hipSuccess) e = hipEventCreateWithFlags(&ctx->na_done_ev, hipEventDisableTiming);
        if (e != hipSuccess) { rc = map_err(e); break; }
    } while (false);
    if (rc != VC_OK) {
        cipher_destroy(ctx);
        return rc;
    }
    *out = ctx;
    return VC_OK;
}

static int locked_call(vc_cipher *ctx, const CallArgs &a) {
    if (!ctx) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    return run_call(ctx, a);
}

int encrypt_frames(vc_cipher *ctx, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                   uint8_t *hashes, uint8_t *const *out, void *stream) {
    if (count && (!frames || !shapes || !hashes || !out)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::Encrypt;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    a.hashes_out = hashes;
    a.out = out;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

int encrypt_frames_noalloc(vc_cipher *ctx, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                           uint8_t *hashes, uint8_t *const *out, void *stream) {
    if (count && (!frames || !shapes || !hashes || !out)) return VC_EINVAL;
    if (!ctx) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::Encrypt;
    a.noalloc = true;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    a.hashes_out = hashes;
    a.out = out;
    a.stream = static_cast<hipStream_t>(stream);
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    ctx->in_noalloc = true;
    const int rc = run_call(ctx, a);
    ctx->in_noalloc = false;
    return rc;
}

int decrypt_frames(vc_cipher *ctx, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                   const uint8_t *hashes, uint8_t *const *out, void *stream) {
    if (count && (!frames || !shapes || !hashes || !out)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::Decrypt;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    a.hashes = hashes;
    a.out = out;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

}  // extern "C"

int vc::call_frames(vc_cipher *ctx, CallKind kind, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                    uint8_t *const *hash_ptrs, uint8_t *const *out, hipStream_t stream) {
    if (count && (!frames || !shapes || !hash_ptrs || (kind != CallKind::Hash && !out))) return VC_EINVAL;
    for (size_t f = 0; f < count; ++f)
        if (!hash_ptrs[f]) return VC_EINVAL;
    CallArgs a{};
    a.op = kind == CallKind::Encrypt         ? Op::Encrypt
           : kind == CallKind::EncryptHashed ? Op::EncryptHashed
           : kind == CallKind::Decrypt       ? Op::Decrypt
                                             : Op::Hash;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    a.hash_ptrs = hash_ptrs;
    a.out = kind == CallKind::Hash ? nullptr : out;
    a.stream = stream;
    return locked_call(ctx, a);
}

extern "C" {

int vc_hash_frames(vc_cipher *ctx, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                   uint8_t *hashes, void *stream) {
    if (count && (!frames || !shapes || !hashes)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::Hash;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    a.hashes_out = hashes;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

int vc_debug_confuse(vc_cipher *ctx, int decrypt, size_t count, const uint8_t *const *in, const vc_shape *shapes,
                     const uint16_t *const *D, const uint8_t *const *B, uint8_t *const *out, void *stream) {
    if (count && (!in || !shapes || !D || !B || !out)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::DebugConfuse;
    a.decrypt = decrypt ? 1 : 0;
    a.count = count;
    a.in = in;
    a.shapes = shapes;
    a.dbgD = D;
    a.dbgB = B;
    a.out = out;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

int vc_debug_keygen(vc_cipher *ctx, size_t count, const vc_shape *shapes, const double *const *IR,
                    uint16_t *const *D, uint8_t *const *B, void *stream) {
    if (count && (!shapes || !IR || !D || !B)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::DebugKeygen;
    a.count = count;
    a.shapes = shapes;
    a.kIR = const_cast<double *const *>(IR);
    a.kD = D;
    a.kB = B;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

int vc_debug_keysched(vc_cipher *ctx, size_t count, const vc_shape *shapes, const uint8_t *hashes,
                      double *const *IR, uint16_t *const *D, uint8_t *const *B, void *stream) {
    if (count && (!shapes || !hashes || !IR || !D || !B)) return VC_EINVAL;
    CallArgs a{};
    a.op = Op::DebugKeysched;
    a.count = count;
    a.shapes = shapes;
    a.hashes = hashes;
    a.kIR = IR;
    a.kD = D;
    a.kB = B;
    a.stream = static_cast<hipStream_t>(stream);
    return locked_call(ctx, a);
}

int cipher_stream_reset(vc_cipher *ctx, uint32_t stream) {
    if (!ctx || stream >= ctx->max_streams) return VC_EINVAL;
    const double st[4] = {ctx->key.x0, ctx->key.y0, ctx->key.z0, ctx->key.w0};
    return cipher_stream_set_state(ctx, stream, st, 0);
}

int cipher_stream_get_state(vc_cipher *ctx, uint32_t stream, double st[4], uint64_t *next_seq) {
    if (!ctx || !st || stream >= ctx->max_streams) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(st, ctx->d_state + 4ull * stream, 4 * sizeof(double), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return map_err(e);
    if (next_seq) *next_seq = ctx->next_seq[stream];
    return VC_OK;
}

int cipher_stream_set_state(vc_cipher *ctx, uint32_t stream, const double st[4], uint64_t next_seq) {
    if (!ctx || !st || stream >= ctx->max_streams) return VC_EINVAL;
    for (int k = 0; k < 4; ++k)
        if (!std::isfinite(st[k])) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    hipError_t e = hipDeviceSynchronize();
    if (e == hipSuccess)
        e = hipMemcpy(ctx->d_state + 4ull * stream, st, 4 * sizeof(double), hipMemcpyHostToDevice);
    if (e != hipSuccess) return map_err(e);
    ctx->next_seq[stream] = next_seq;
    return VC_OK;
}

int cipher_status(vc_cipher *ctx, void *stream) {
    if (!ctx) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
    int flags = 0;
    if (e == hipSuccess) e = hipMemcpy(&flags, ctx->d_flags, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return map_err(e);
    if (flags) {
        const int zero = 0;
        e = hipMemcpy(ctx->d_flags, &zero, sizeof(int), hipMemcpyHostToDevice);
        if (e != hipSuccess) return map_err(e);
        return VC_ENONFINITE;
    }
    return VC_OK;
}

int vc_profile_enable(vc_cipher *ctx, int enable) {
    if (!ctx) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->profile = enable != 0;
    return VC_OK;
}

int vc_profile_read(vc_cipher *ctx, int kernel_id, double *total_ms, uint64_t *launches) {
    if (!ctx || kernel_id < 0 || kernel_id >= K_COUNT) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    hipError_t e = drain_profile(ctx);
    if (e != hipSuccess) return map_err(e);
    if (total_ms) *total_ms = ctx->acc_ms[kernel_id];
    if (launches) *launches = ctx->acc_n[kernel_id];
    return VC_OK;
}

int vc_profile_reset(vc_cipher *ctx) {
    if (!ctx) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    hipError_t e = drain_profile(ctx);
    for (int k = 0; k < K_COUNT; ++k) {
        ctx->acc_ms[k] = 0;
        ctx->acc_n[k] = 0;
    }
    return map_err(e);
}

int vc_set_overlap(vc_cipher *ctx, uint32_t parts, uint32_t side_streams, uint32_t scratch_slots) {
    if (!ctx || parts < 1 || parts > 64 || side_streams > kMaxSide || scratch_slots < 1 || scratch_slots > kMaxSlots)
        return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    if (scratch_slots != ctx->nslots) {
        // slot boundaries move: let all work that uses the scratch finish
        const hipError_t e = hipDeviceSynchronize();
        if (e != hipSuccess) return map_err(e);
        for (auto &row : ctx->slot_live)
            for (bool &b : row) b = false;
        ctx->nslots = scratch_slots;
        ctx->slot_next = 0;
    }
    ctx->parts = parts;
    ctx->nside = side_streams;
    ctx->side_base = 0;
    return VC_OK;
}

int vc_autotune(vc_cipher *ctx, int decrypt, uint32_t w, uint32_t h, uint32_t frames, uint32_t *strip_out,
                uint32_t *threads_out) {
    if (!ctx || frames < 1 || frames > 4096) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    const vc_shape shape{w, h, 3, 0, 0};
    int rc = check_shape(ctx, shape, decrypt ? 1 : 0, false);
    if (rc) return rc;
    const uint64_t L = frame_bytes(shape), ND = 3ull * h + 3ull * w;
    const uint64_t Lp = align_up(L, 256), Dp = align_up(2 * ND, 256);
    uint8_t *buf = nullptr;
    FrameDesc *d_desc = nullptr;
    hipStream_t st = nullptr;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const uint64_t total = frames * (4 * Lp + Dp);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&buf), total);
    if (e == hipSuccess) e = hipMalloc(reinterpret_cast<void **>(&d_desc), sizeof(FrameDesc) * frames);
    if (e == hipSuccess) e = hipStreamCreateWithFlags(&st, hipStreamNonBlocking);
    if (e == hipSuccess) e = hipEventCreate(&e0);
    if (e == hipSuccess) e = hipEventCreate(&e1);
    uint32_t best_strip = 0, best_threads = 0;
    if (e == hipSuccess) {
        // frames, keystream and an intermediate image (contents do not matter:
        // the kernels are data-oblivious); distances pseudorandom
        std::vector<FrameDesc> desc(frames);
        std::vector<uint16_t> D(ND);
        uint32_t x = 0x9E3779B9u;
        for (auto &v : D) {
            x = x * 1664525u + 1013904223u;
            v = static_cast<uint16_t>(x >> 16);
        }
        for (uint32_t f = 0; f < frames && e == hipSuccess; ++f) {
            uint8_t *base = buf + f * (4 * Lp + Dp);
            desc[f] = FrameDesc{base, base + Lp, nullptr, nullptr, reinterpret_cast<uint16_t *>(base + 4 * Lp),
                                base + 2 * Lp, base + 3 * Lp, w, h, L, 0, 0};
            e = hipMemcpyAsync(base + 4 * Lp, D.data(), 2 * ND, hipMemcpyHostToDevice, st);
        }
        if (e == hipSuccess) e = hipMemsetAsync(buf, 0x5A, frames * (4 * Lp), st);
        if (e == hipSuccess)
            e = hipMemcpyAsync(d_desc, desc.data(), sizeof(FrameDesc) * frames, hipMemcpyHostToDevice, st);
        if (e == hipSuccess) e = hipStreamSynchronize(st);
        // buffers are 256-byte aligned: the alignment class is the rows'
        const int align = (w % 16 == 0) ? 2 : (w % 4 == 0) ? 1 : 0;
        // candidate strips: bytes of a row (two-pass) or pixels (single pass)
        const uint32_t cap = ctx->passes == 2
                                 ? std::max<uint32_t>(4, 1u << (32 - __builtin_clz(std::max<uint32_t>(3 * w, 2) - 1)))
                                 : std::max<uint32_t>(4, (w + 3) / 4 * 4);
        const uint32_t widest = ctx->passes == 2 ? 128 : 64;
        float best = 1e30f;
        for (uint32_t wt = 4; wt <= widest && e == hipSuccess; wt *= 2) {
            if (wt > cap) break;
            const uint32_t lds = ctx->passes == 2 ? shift_col_lds_bytes(h, wt) : confuse_lds_bytes(decrypt, h, wt);
            if (lds > ctx->lds_limit) continue;
            for (uint32_t nt : {256u, 512u, 1024u}) {
                ConfuseTuning t;
                t.strip = wt;
                t.threads = nt;
                t.xcd_map = ctx->xcd_map;
                // the strip-tiled pass only (the row pass does not depend on the
                // tiling), on the layout that the strip implies
                if (ctx->passes == 2) {
                    const uint32_t ls = shift_xstrip(w, wt, align, ctx->lds_limit);
                    if (desc[0].xstrip != ls) {
                        for (auto &dd : desc) dd.xstrip = ls;
                        e = hipMemcpyAsync(d_desc, desc.data(), sizeof(FrameDesc) * frames, hipMemcpyHostToDevice,
                                           st);
                        if (e == hipSuccess) e = hipStreamSynchronize(st);
                        if (e != hipSuccess) break;
                    }
                }
                auto run = [&] {
                    if (ctx->passes == 2)
                        return launch_shift(decrypt, decrypt ? 0 : 1, d_desc, 0, frames, w, h, align, t,
                                            ctx->lds_limit, st);
                    return launch_confuse(decrypt, d_desc, 0, frames, w, h, align >= 1, t, st);
                };
                e = run();  // warm-up
                if (e == hipSuccess) e = hipEventRecord(e0, st);
                for (int r = 0; r < 3 && e == hipSuccess; ++r) e = run();
                if (e == hipSuccess) e = hipEventRecord(e1, st);
                if (e == hipSuccess) e = hipEventSynchronize(e1);
                float ms = 0.f;
                if (e == hipSuccess) e = hipEventElapsedTime(&ms, e0, e1);
                if (e == hipSuccess && ms < best) {
                    best = ms;
                    best_strip = wt;
                    best_threads = nt;
                }
            }
        }
    }
    if (e1) (void)hipEventDestroy(e1);
    if (e0) (void)hipEventDestroy(e0);
    if (st) (void)hipStreamDestroy(st);
    if (d_desc) (void)hipFree(d_desc);
    if (buf) (void)hipFree(buf);
    if (e != hipSuccess) return map_err(e);
    if (!best_strip) return VC_EINVAL;
    ctx->tuned[std::make_tuple(w, h, decrypt ? 1 : 0, ctx->passes)] = {best_strip, best_threads};
    if (strip_out) *strip_out = best_strip;
    if (threads_out) *threads_out = best_threads;
    return VC_OK;
}

}  // extern "C"

// ---- prepared batches ----

struct vc_batch {
    vc_cipher *ctx = nullptr;
    int mode = VC_PREP_ENCRYPT;
    int decrypt = 0;
    bool two_pass = true;
    uint32_t count = 0;
    uint8_t *d_mem = nullptr;  // descriptors, then the batch's scratch
    const FrameDesc *d_desc = nullptr;
    const StreamRun *d_runs = nullptr;
    const ChainRec *d_order = nullptr;
    std::vector<Chunk> chunks;
    std::vector<std::vector<ConfuseTuning>> tiling;  // per chunk, per shape group
    std::map<uint32_t, uint64_t> frames_per_stream;
};

namespace {

void batch_free(vc_batch *b) {
    if (b->d_mem) (void)hipFree(b->d_mem);
    delete b;
}

}  // namespace

extern "C" {

int vc_batch_prepare(vc_cipher *ctx, int mode, size_t count, const uint8_t *const *frames, const vc_shape *shapes,
                     uint8_t *hashes, uint8_t *const *out, vc_batch **batch) {
    if (batch) *batch = nullptr;
    const bool hash_only = mode == VC_PREP_HASH;
    if (mode != VC_PREP_ENCRYPT && mode != VC_PREP_DECRYPT && !hash_only && mode != VC_PREP_ENCRYPT_HASHED)
        return VC_EINVAL;
    if (!ctx || !batch || count == 0 || count > 0xFFFFFFFFull || !frames || !shapes || !hashes ||
        (!out && !hash_only))
        return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    const int dec = mode == VC_PREP_DECRYPT ? 1 : 0;
    // a hash batch runs only the frame hashes: no chain, no scratch
    const bool two_pass = ctx->passes == 2 && !hash_only;
    const uint32_t n = ctx->key.n;
    std::map<uint32_t, uint64_t> last_seq;
    uint64_t need = 0;
    for (size_t f = 0; f < count; ++f) {
        const vc_shape &s = shapes[f];
        const int rc = check_shape(ctx, s, dec, true);
        if (rc) return rc;
        if (!frames[f]) return VC_EINVAL;
        if (hash_only) continue;
        const uint64_t L = frame_bytes(s);
        if (!out[f] || overlaps(frames[f], L, out[f], L)) return VC_EINVAL;
        if (s.stream >= ctx->max_streams) return VC_EINVAL;
        auto it = last_seq.find(s.stream);
        if (it != last_seq.end() && s.seq <= it->second) return VC_EORDER;
        last_seq[s.stream] = s.seq;
        need += scratch_need(s, n, true, two_pass);
    }
    // the kernels read and write the hash buffer in place
    if (!reachable(hashes, 32 * count)) return VC_EINVAL;
    vc_batch *b = new (std::nothrow) vc_batch();
    if (!b) return VC_ENOMEM;
    b->ctx = ctx;
    b->mode = mode;
    b->decrypt = dec;
    b->two_pass = two_pass;
    b->count = static_cast<uint32_t>(count);
    if (!hash_only)
        for (size_t f = 0; f < count; ++f) b->frames_per_stream[shapes[f].stream] += 1;
    CallArgs a{};
    a.op = mode == VC_PREP_DECRYPT         ? Op::Decrypt
           : mode == VC_PREP_HASH          ? Op::Hash
           : mode == VC_PREP_ENCRYPT_HASHED ? Op::EncryptHashed
                                            : Op::Encrypt;
    a.count = count;
    a.in = frames;
    a.shapes = shapes;
    if (mode == VC_PREP_DECRYPT || mode == VC_PREP_ENCRYPT_HASHED) a.hashes = hashes;
    else a.hashes_out = hashes;
    a.out = hash_only ? nullptr : out;
    // descriptors first (at most one run and one chain record per frame),
    // then one span of scratch for every frame
    const size_t desc_max = align_up(sizeof(FrameDesc) * count, 256) + align_up(sizeof(StreamRun) * count, 256) +
                            align_up(sizeof(ChainRec) * count, 256);
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&b->d_mem), desc_max + need);
    if (e != hipSuccess) {
        batch_free(b);
        return map_err(e);
    }
    Plan P;
    build_plan(ctx, a, !hash_only, two_pass, !hash_only, !hash_only, dec, need, 1,
               [&](uint32_t) { return b->d_mem + desc_max; }, P);
    const size_t desc_bytes = align_up(sizeof(FrameDesc) * count, 256);
    const size_t runs_bytes = align_up(sizeof(StreamRun) * count, 256);
    e = hipMemcpy(b->d_mem, P.desc.data(), sizeof(FrameDesc) * count, hipMemcpyHostToDevice);
    if (e == hipSuccess && !P.runs.empty())
        e = hipMemcpy(b->d_mem + desc_bytes, P.runs.data(), sizeof(StreamRun) * P.runs.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && !P.order.empty())
        e = hipMemcpy(b->d_mem + desc_bytes + runs_bytes, P.order.data(), sizeof(ChainRec) * P.order.size(),
                      hipMemcpyHostToDevice);
    if (e != hipSuccess) {
        batch_free(b);
        return map_err(e);
    }
    b->d_desc = reinterpret_cast<const FrameDesc *>(b->d_mem);
    b->d_runs = reinterpret_cast<const StreamRun *>(b->d_mem + desc_bytes);
    b->d_order = reinterpret_cast<const ChainRec *>(b->d_mem + desc_bytes + runs_bytes);
    if (!hash_only) b->chunks = P.chunks;
    for (const Chunk &ch : b->chunks) {
        std::vector<ConfuseTuning> t;
        for (const Group &gr : ch.groups) t.push_back(choose_tiling(ctx, dec, gr.w, gr.h));
        b->tiling.push_back(std::move(t));
    }
    *batch = b;
    return VC_OK;
}

int vc_batch_launch(vc_batch *b, void *stream) {
    if (!b) return VC_EINVAL;
    vc_cipher *ctx = b->ctx;
    std::lock_guard<std::mutex> lk(ctx->mu);
    DeviceGuard g(ctx->device);
    if (!g.ok) return VC_EDEVICE;
    const hipStream_t s = static_cast<hipStream_t>(stream);
    const uint32_t n = ctx->key.n;
    hipError_t e = hipSuccess;
    if (b->mode == VC_PREP_ENCRYPT || b->mode == VC_PREP_HASH) e = launch_sha256_subframes(b->d_desc, b->count, n, s);
    const hipStream_t ws = s;
    for (size_t ci = 0; ci < b->chunks.size() && e == hipSuccess; ++ci) {
        const Chunk &ch = b->chunks[ci];
        e = launch_lhcs_chain(b->d_runs + ch.run_begin, b->d_order, ch.run_end - ch.run_begin, ctx->d_state, n,
                              ctx->key.gamma, ctx->d_flags, s);
        if (e == hipSuccess)
            e = launch_lhcs_keygen(b->d_desc + ch.desc_begin, ch.desc_end - ch.desc_begin, n, ctx->key.gamma,
                                   ctx->d_flags, ws);
        for (size_t gi = 0; gi < ch.groups.size() && e == hipSuccess; ++gi) {
            const Group &gr = ch.groups[gi];
            const ConfuseTuning &t = b->tiling[ci][gi];
            if (!b->two_pass) {
                e = launch_confuse(b->decrypt, b->d_desc, gr.first, gr.count, gr.w, gr.h, gr.align >= 1, t, ws);
            } else {
                for (int pass = 0; pass < 2 && e == hipSuccess; ++pass)
                    e = launch_shift(b->decrypt, pass, b->d_desc, gr.first, gr.count, gr.w, gr.h, gr.align, t,
                                     ctx->lds_limit, ws);
            }
        }
    }
    if (e != hipSuccess) return map_err(e);
    for (const auto &kv : b->frames_per_stream) ctx->next_seq[kv.first] += kv.second;
    return VC_OK;
}

void vc_batch_destroy(vc_batch *b) {
    if (!b) return;
    DeviceGuard g(b->ctx->device);
    (void)hipDeviceSynchronize();
    batch_free(b);
}

}  // extern "C"

namespace {

// Device copy of the frame table (and an optional host array of uint32
// pairs), for the statistics entry points.  Synchronous upload; freed by
// the destructor after the stream has been synchronised.
struct StatUpload {
    StatFrame *frames = nullptr;
    uint32_t *pairs = nullptr;
    ~StatUpload() {
        if (pairs) (void)hipFree(pairs);
        if (frames) (void)hipFree(frames);
    }
};

int stat_frames(size_t count, const uint8_t *const *frames, const vc_shape *shapes, std::vector<StatFrame> &out) {
    if (!frames || !shapes || count > 0xFFFFFFFFull) return VC_EINVAL;
    out.resize(count);
    for (size_t f = 0; f < count; ++f) {
        const vc_shape &s = shapes[f];
        if (!frames[f] || s.c != 3 || s.w < 1 || s.h < 1 || s.w > kMaxDim || s.h > kMaxDim) return VC_EINVAL;
        out[f] = StatFrame{frames[f], s.w, s.h};
    }
    return VC_OK;
}

hipError_t upload(StatUpload &u, const std::vector<StatFrame> &fr, const uint32_t *pairs, size_t npairs_words) {
    hipError_t e = hipMalloc(reinterpret_cast<void **>(&u.frames), sizeof(StatFrame) * fr.size());
    if (e == hipSuccess) e = hipMemcpy(u.frames, fr.data(), sizeof(StatFrame) * fr.size(), hipMemcpyHostToDevice);
    if (e == hipSuccess && pairs && npairs_words) {
        e = hipMalloc(reinterpret_cast<void **>(&u.pairs), 4 * npairs_words);
        if (e == hipSuccess) e = hipMemcpy(u.pairs, pairs, 4 * npairs_words, hipMemcpyHostToDevice);
    }
    return e;
}

}  // namespace

extern "C" {

int vc_frame_histograms(size_t count, const uint8_t *const *frames, const vc_shape *shapes, uint32_t *hist,
                        void *stream) {
    if (count == 0) return VC_OK;
    if (!hist) return VC_EINVAL;
    std::vector<StatFrame> fr;
    int rc = stat_frames(count, frames, shapes, fr);
    if (rc) return rc;
    uint64_t max_bytes = 0;
    for (auto &f : fr) max_bytes = std::max<uint64_t>(max_bytes, 3ull * f.w * f.h);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    StatUpload u;
    hipError_t e = upload(u, fr, nullptr, 0);
    if (e == hipSuccess) e = hipMemsetAsync(hist, 0, sizeof(uint32_t) * 3 * 256 * count, s);
    if (e == hipSuccess) e = launch_frame_histograms(u.frames, static_cast<uint32_t>(count), max_bytes, hist, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return map_err(e);
}

int vc_block_histograms(size_t count, const uint8_t *const *frames, const vc_shape *shapes, uint32_t blocks,
                        uint32_t block_w, uint32_t block_h, const uint32_t *origins, uint32_t *hist, void *stream) {
    if (count == 0 || blocks == 0) return VC_OK;
    if (!hist || !origins || block_w < 1 || block_h < 1) return VC_EINVAL;
    std::vector<StatFrame> fr;
    int rc = stat_frames(count, frames, shapes, fr);
    if (rc) return rc;
    for (size_t f = 0; f < count; ++f)
        for (uint32_t m = 0; m < blocks; ++m) {
            const uint32_t r = origins[2 * (f * blocks + m)], c = origins[2 * (f * blocks + m) + 1];
            if (static_cast<uint64_t>(r) + block_h > fr[f].h || static_cast<uint64_t>(c) + block_w > fr[f].w)
                return VC_EINVAL;
        }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    StatUpload u;
    hipError_t e = upload(u, fr, origins, 2 * count * blocks);
    if (e == hipSuccess)
        e = launch_block_histograms(u.frames, static_cast<uint32_t>(count), blocks, block_w, block_h, u.pairs, hist, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return map_err(e);
}

int vc_pair_moments(size_t count, const uint8_t *const *frames, const vc_shape *shapes, uint32_t npairs,
                    const uint32_t *positions, uint64_t *moments, void *stream) {
    if (count == 0) return VC_OK;
    if (!moments || (positions && npairs == 0)) return VC_EINVAL;
    std::vector<StatFrame> fr;
    int rc = stat_frames(count, frames, shapes, fr);
    if (rc) return rc;
    uint64_t max_pos = 0;
    for (size_t f = 0; f < count; ++f) {
        if (positions) {
            for (uint32_t i = 0; i < npairs; ++i) {
                const uint32_t r = positions[2 * (f * npairs + i)], c = positions[2 * (f * npairs + i) + 1];
                if (static_cast<uint64_t>(r) + 1 >= fr[f].h || static_cast<uint64_t>(c) + 1 >= fr[f].w)
                    return VC_EINVAL;
            }
            max_pos = npairs;
        } else {
            max_pos = std::max<uint64_t>(max_pos, static_cast<uint64_t>(fr[f].h - 1) * (fr[f].w - 1));
        }
    }
    const hipStream_t s = static_cast<hipStream_t>(stream);
    StatUpload u;
    hipError_t e = upload(u, fr, positions, positions ? 2 * count * npairs : 0);
    if (e == hipSuccess) e = hipMemsetAsync(moments, 0, sizeof(uint64_t) * 45 * count, s);
    if (e == hipSuccess)
        e = launch_pair_moments(u.frames, static_cast<uint32_t>(count), max_pos, npairs, u.pairs,
                                reinterpret_cast<unsigned long long *>(moments), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return map_err(e);
}

int vc_frame_diff(size_t count, const uint8_t *const *a, const uint8_t *const *b, const vc_shape *shapes,
                  uint64_t *out, void *stream) {
    if (count == 0) return VC_OK;
    if (!out || !b) return VC_EINVAL;
    std::vector<StatFrame> fa, fb;
    int rc = stat_frames(count, a, shapes, fa);
    if (rc) return rc;
    rc = stat_frames(count, b, shapes, fb);
    if (rc) return rc;
    uint64_t max_bytes = 0;
    for (auto &f : fa) max_bytes = std::max<uint64_t>(max_bytes, 3ull * f.w * f.h);
    const hipStream_t s = static_cast<hipStream_t>(stream);
    StatUpload ua, ub;
    hipError_t e = upload(ua, fa, nullptr, 0);
    if (e == hipSuccess) e = upload(ub, fb, nullptr, 0);
    if (e == hipSuccess) e = hipMemsetAsync(out, 0, sizeof(uint64_t) * 12 * count, s);
    if (e == hipSuccess)
        e = launch_frame_diff(ua.frames, ub.frames, static_cast<uint32_t>(count), max_bytes,
                              reinterpret_cast<unsigned long long *>(out), s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    return map_err(e);
}

int vc_pointer_reachable(const void *p, size_t bytes) { return vc::reachable(p, bytes) ? 1 : 0; }

int vc_bandwidth_probe(int kind, const uint8_t *a, const uint8_t *b, uint8_t *out, size_t bytes, void *stream) {
    if ((kind != 0 && kind != 1) || !a || !out || (kind == 1 && !b) || bytes % 16) return VC_EINVAL;
    if ((reinterpret_cast<uintptr_t>(a) | reinterpret_cast<uintptr_t>(out) |
         (kind == 1 ? reinterpret_cast<uintptr_t>(b) : 0)) & 15)
        return VC_EINVAL;
    return map_err(launch_stream_probe(kind, a, b, out, bytes, static_cast<hipStream_t>(stream)));
}

uint32_t vc_max_frame_height(const vc_cipher *ctx) {
    if (!ctx) return 0;
    // the largest h for which both directions have a strip width that fits
    auto ok = [&](uint32_t h) {
        if (ctx->passes == 2) return shift_max_strip(h, ctx->lds_limit) != 0;
        return confuse_max_strip(0, h, ctx->lds_limit) != 0 && confuse_max_strip(1, h, ctx->lds_limit) != 0;
    };
    uint32_t lo = 0, hi = kMaxDim;  // ok(lo) (or lo == 0), answer in [lo, hi]
    while (lo < hi) {
        const uint32_t mid = lo + (hi - lo + 1) / 2;
        if (ok(mid)) lo = mid;
        else hi = mid - 1;
    }
    return lo;
}

int vc_set_confusion_passes(vc_cipher *ctx, uint32_t passes) {
    if (!ctx || (passes != 1 && passes != 2)) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->passes = static_cast<int>(passes);
    return VC_OK;
}

size_t vc_scratch_per_frame(uint32_t w, uint32_t h, uint32_t n) {
    vc_shape s{w, h, 3, 0, 0};
    return static_cast<size_t>(scratch_need(s, n, true, true));
}

int vc_set_tuning(vc_cipher *ctx, uint32_t strip_width, uint32_t threads, int xcd_map) {
    if (!ctx) return VC_EINVAL;
    if (strip_width && (strip_width < 4 || strip_width > 128 || (strip_width & (strip_width - 1))))
        return VC_EINVAL;
    if (threads && threads != 256 && threads != 512 && threads != 1024) return VC_EINVAL;
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->strip = strip_width;
    ctx->threads = threads;
    ctx->xcd_map = xcd_map ? 1 : 0;
    return VC_OK;
}

}  // extern "C"
