// Host-side internal interfaces between the translation units of libmh.
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

#include "mh.h"

namespace mh {

struct NodeRec;

// Bump allocator over a caller-provided workspace (256-byte aligned pieces).
struct Arena {
    char* base = nullptr;
    size_t size = 0;
    size_t used = 0;
    bool overflow = false;

    Arena(void* p, size_t n) : base(static_cast<char*>(p)), size(n) {}

    template <typename T>
    T* take(size_t count) {
        size_t off = (used + 255) & ~size_t(255);
        size_t bytes = count * sizeof(T);
        used = off + bytes;
        if (used > size || base == nullptr) {
            overflow = true;
            return nullptr;
        }
        return reinterpret_cast<T*>(base + off);
    }
};

// Counting pass: same sequence of take() calls with no memory behind it
// (every piece comes back null).
struct Sizer {
    size_t used = 0;
    template <typename T>
    T* take(size_t count) {
        used = ((used + 255) & ~size_t(255)) + count * sizeof(T);
        return nullptr;
    }
};

// A range of u64 words for a zeroing kernel to clear (n = 0: none).
struct ZeroRange {
    uint64_t* p = nullptr;
    int64_t n = 0;
};

#define MH_HIP_TRY(expr)                              \
    do {                                              \
        hipError_t e_ = (expr);                       \
        if (e_ != hipSuccess) return MH_EHIP;         \
    } while (0)

// ---- device facts, queried once per device (and kernel) and kept ----
// Compute units of the current device (256 if the query fails).
int device_cus();
// Blocks of `kernel` with `threads` threads that one CU holds at once (>= 1).
int blocks_per_cu(const void* kernel, int threads);
template <typename K>
int64_t resident_blocks(K kernel, int threads) {
    return (int64_t)device_cus() * blocks_per_cu(reinterpret_cast<const void*>(kernel), threads);
}

// ---- exclusive scans: out[0..n] with out[n] = total (in may alias out) ----
size_t scan_workspace_bytes(int64_t n);
mh_status scan_exclusive_u64(const uint64_t* in, uint64_t* out, int64_t n, void* ws, size_t ws_bytes,
                             hipStream_t stream);
mh_status scan_exclusive_u32(const uint32_t* in, uint32_t* out, int64_t n, void* ws, size_t ws_bytes,
                             hipStream_t stream);

// Single-kernel variant (decoupled look-back, mh_lookback.hpp) for sums below
// 2^62; state: lb_tiles(n) u64 words, zero at launch (zeroed by an earlier
// kernel); samples (optional, lb_samples(n) words): out[256 k]; err (device,
// not null) receives MH_EHIP if a look-back stalls.
mh_status scan_exclusive_u64_onepass(const uint64_t* in, uint64_t* out, int64_t n, uint64_t* state,
                                     uint64_t* samples, int32_t* err, hipStream_t stream);

// ---- radix sort of 64-bit keys with distinct 32-bit payloads ----
// Passed split: hi[i] = key >> 32 (the radix key, kRadixPasses passes of 8
// bits) and pay[i] = (key & 0xFFFFFFFF) << 32 | payload; afterwards the pairs
// ascend by (key, payload).
constexpr int kRadixPasses = 4;
// Copies of the digit histograms: enough that no address takes more than a few
// dozen of the counting kernel's atomics, few enough that each pass sums them
// with one round of loads.
constexpr int kRadixHistCopies = 4;
size_t radix_workspace_bytes(int64_t n);
// Zeroes the sort's scratch (in ws) and returns its histogram array for the
// counting kernel that writes hi and pay: kRadixHistCopies copies of
// kRadixPasses x 256 counts of the bytes of hi (copy c, pass p, digit d at
// [(c * kRadixPasses + p) * 256 + d]); a counting block adds into copy
// blockIdx % kRadixHistCopies.
// e1, e2: further ranges of u64 words zeroed by the same kernel.  x (and y)
// non-null: the same kernel also takes the least and largest sort key of every
// tile of the node parameters, for a first pass that makes the keys itself.
mh_status radix_prepare(void* ws, size_t ws_bytes, int64_t n, uint32_t** hist, hipStream_t stream,
                        ZeroRange e1 = {}, ZeroRange e2 = {}, const double* x = nullptr, const double* y = nullptr);
// Sorts hi[0..n) / pay[0..n) using alt buffers of the same size (the result
// ends in hi / pay); the histograms must hold the counts.  err (optional,
// device) receives MH_EHIP if a look-back or exchange ever stalls.
// x (and y) non-null: the first pass makes the keys itself from the node
// parameters (z = x or x y, checks raising MH_EINVAL into err) and counts the
// later passes' digits, so hi / pay need no preparation and the histograms
// only need to be zero; allowed when radix_prepares_keys(n), with the same x
// and y given to radix_prepare.  The keys are then sorted less their least
// value (*kbase, a device word, receives it: hi ends as key >> 32 minus
// *kbase) by as many passes as their spread needs, and *tile_mass receives
// the column masses floor(z 2^32) summed per tile of 4096 nodes (device, one
// word per tile: their total is the masses' sum in any order); otherwise both
// are null.
bool radix_prepares_keys(int64_t n);
mh_status radix_sort_split64(uint32_t* hi, uint64_t* pay, uint32_t* hi_alt, uint64_t* pay_alt, int64_t n,
                             void* ws, size_t ws_bytes, int32_t* err, hipStream_t stream,
                             const double* x = nullptr, const double* y = nullptr,
                             const uint32_t** kbase = nullptr, const uint64_t** tile_mass = nullptr);

// ---- sampler pieces ----
struct SortedView {
    int32_t* perm = nullptr;
    double* zs = nullptr;
    double* ys = nullptr;  // weighted only
    double* c = nullptr;   // weighted only
};

size_t order_workspace_bytes(int64_t n);
// The sorted order before records are made from it (see order_nodes).
struct SortedKeys {
    const uint32_t* keys = nullptr;       // high halves of the sort keys, less *kbase
    const uint64_t* vals = nullptr;       // low half << 32 | node id
    const uint32_t* kbase = nullptr;      // device word
    const uint64_t* tile_mass = nullptr;  // column masses summed per tile of 4096 nodes (input order)
    int64_t tiles = 0;
};
// Writes the order either as packed records (node != null: z and id; nseg is
// left for the plan) or as separate perm / zs arrays.  mass_prefix (optional,
// n + 1 entries): P[r] = sum of the column masses floor(z 2^32) (2^32 for
// z >= 1) over ranks < r, P[n] = total; with node records this is computed in
// the same pass, with the look-back state mass_state (lb_tiles(n) words that
// must be zero when this call's first kernel has run: pass them as e1 or
// e2), and then mass_samples (optional, lb_samples(n) words) receives
// P[256 k] and z_samples (optional, (n - 1) / 256 + 1 values) z[256 k].  check_square: the largest z squared must be finite (one node
// set, where it is the largest t).  e1, e2: u64 words zeroed by the first
// kernel (look-back state of later steps, counters).  sorted (optional):
// when the sort made its keys from x (radix_prepares_keys), the order stops
// there, leaving the sorted arrays (in ws) in *sorted for a caller that makes
// the records itself; otherwise sorted->keys stays null and the order is
// finished as above.
mh_status order_nodes(const double* x, const double* y, int64_t n, int32_t* perm, double* zs, double* ys,
                      NodeRec* node, int32_t* status, uint64_t* mass_prefix, uint64_t* mass_state,
                      uint64_t* mass_samples, double* z_samples, void* ws, size_t ws_bytes, hipStream_t stream,
                      bool check_square = true, ZeroRange e1 = {}, ZeroRange e2 = {}, SortedKeys* sorted = nullptr);

size_t bound_workspace_bytes(int64_t n);
mh_status bound_suffix_top2(const double* ys, int64_t n, double* c, int32_t* status, void* ws, size_t ws_bytes,
                            hipStream_t stream);

}  // namespace mh
