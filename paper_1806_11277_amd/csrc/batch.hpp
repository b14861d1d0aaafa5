// Launches over several subdomains at once.
//
// Every kernel of the cycle and of the DD transfers is written as a device body
// taking its block index as a VB (block index, block count) plus two entry
// points: NAME(args), one launch as usual, and NAME_batch(Batch), one launch for
// up to kMaxBatch subdomains whose argument packs travel by value in the
// kernel arguments (so a captured graph keeps them).  The batch grid is the
// subdomains' x-grids laid end to end (a flat (subdomain, block) list: uneven
// subdomains waste no block), and the largest y and z extents, where a block
// beyond its own subdomain's y or z extent returns at once.
//
// EHH_LAUNCHK(BYTES, NAME, (template args), GRID, BLOCK, SHMEM, STREAM, args...)
// launches NAME<template args>(args...) -- or, while the calling thread records
// (batch_recording()), records the launch with its argument pack so that the
// same launch of several subdomains can be merged into one NAME_batch launch.
#pragma once

#include <hip/hip_runtime.h>

#include <cstring>
#include <functional>

#include "common.hpp"
#include "launchlog.hpp"

namespace ehh {

// Workgroups are dealt to the 8 XCDs round-robin (linear id mod 8), and each XCD
// has its own L2.  Renumbering so that every XCD receives one contiguous range
// of logical blocks keeps the rows above and below a block's cells (stencil
// neighbours) in the same L2.  Bijective for any block count.
EHH_HD inline int64_t xcd_block(int64_t bid, int64_t nb) {
    constexpr int64_t X = 8;
    const int64_t q = nb / X, rem = nb % X;
    const int64_t xcd = bid % X, local = bid / X;
    return xcd < rem ? xcd * (q + 1) + local : rem * (q + 1) + (xcd - rem) * q + local;
}

// The block index a kernel body sees (after the XCD renumbering where the
// kernel uses it) and the number of blocks of its own launch or subdomain.
struct VB {
    unsigned x, n;
};

// Aggregate tuple of kernel arguments (trivially copyable, so it can travel in
// the kernel arguments).
template <class... A> struct Pack;
template <> struct Pack<> {};
template <class H, class... R> struct Pack<H, R...> {
    H h;
    Pack<R...> r;
};
template <class... P> struct PackAs;
template <> struct PackAs<> {
    static EHH_HD Pack<> make() { return Pack<>{}; }
};
template <class H, class... R> struct PackAs<H, R...> {
    template <class A, class... B> static EHH_HD Pack<H, R...> make(A&& a, B&&... b) {
        return Pack<H, R...>{static_cast<H>(a), PackAs<R...>::make(static_cast<B&&>(b)...)};
    }
};
// Pack of a kernel's parameter types, from its function type
template <class K> struct PackOf;
template <class... P> struct PackOf<void (*)(P...)> {
    using type = Pack<P...>;
    using as = PackAs<P...>;
};
template <class F, class... D> EHH_DEV void call_pack(F&& f, const Pack<>&, const D&... d) { f(d...); }
template <class F, class H, class... R, class... D>
EHH_DEV void call_pack(F&& f, const Pack<H, R...>& p, const D&... d) {
    call_pack(f, p.r, d..., p.h);
}

constexpr int kMaxBatch = 8;
template <class PK> struct Batch {
    int n;
    unsigned first[kMaxBatch + 1];   // first flat block of each subdomain (prefix)
    unsigned gy[kMaxBatch], gz[kMaxBatch];
    PK arg[kMaxBatch];
};

// Subdomain s and body block index of this block of a batch launch; false for a
// block beyond its subdomain's y or z extent.
template <bool XCD, class PK> EHH_DEV bool batch_block(const Batch<PK>& b, VB& vb, int& s) {
    const unsigned g = XCD ? (unsigned)xcd_block(blockIdx.x, gridDim.x) : blockIdx.x;
    int k = 0;
    while (k + 1 < b.n && g >= b.first[k + 1]) ++k;
    if (blockIdx.y >= b.gy[k] || blockIdx.z >= b.gz[k]) return false;
    vb.x = g - b.first[k];
    vb.n = b.first[k + 1] - b.first[k];
    s = k;
    return true;
}
template <bool XCD> EHH_DEV VB single_block() {
    return VB{XCD ? (unsigned)xcd_block(blockIdx.x, gridDim.x) : blockIdx.x, gridDim.x};
}

// ---- recording (host)
struct BatchRec {
    const void* kernel;                 // the single-launch entry point (identity)
    const void* batch_kernel;           // its NAME_batch instance for this pack type
    dim3 grid, block;
    size_t shmem;
    LaunchBytes bytes;
    std::vector<char> pack;             // the argument pack's bytes
    // launches recs (same kernel, one per subdomain, at most kMaxBatch) as one
    // batch launch on stream s
    hipError_t (*launch)(const BatchRec* const* recs, int n, hipStream_t s);
};
bool batch_recording();
void batch_record(BatchRec&& r);

template <class PK>
hipError_t launch_batch_pack(const BatchRec* const* recs, int n, hipStream_t s) {
    static_assert(sizeof(Batch<PK>) <= 4096, "batch arguments exceed the kernel argument space");
    Batch<PK> b;
    std::memset(&b, 0, sizeof(b));
    b.n = n;
    unsigned gy = 1, gz = 1, gx = 0;
    LaunchBytes lb;
    for (int i = 0; i < n; ++i) {
        b.first[i] = gx;
        gx += recs[i]->grid.x;
        b.gy[i] = recs[i]->grid.y;
        b.gz[i] = recs[i]->grid.z;
        gy = gy > recs[i]->grid.y ? gy : recs[i]->grid.y;
        gz = gz > recs[i]->grid.z ? gz : recs[i]->grid.z;
        std::memcpy(&b.arg[i], recs[i]->pack.data(), sizeof(PK));
        lb.mine += recs[i]->bytes.mine;
        lb.model += recs[i]->bytes.model;
    }
    b.first[n] = gx;
    const dim3 grid(gx, gy, gz), block = recs[0]->block;
    const size_t sh = recs[0]->shmem;
    const void* k = recs[0]->batch_kernel;
    void* args[] = {&b};
    hipError_t e = hipLaunchKernel(k, grid, block, args, sh, s);
    if (e == hipSuccess && launch_log_on())
        launch_log_add(k, lb, [b, k, grid, block, sh](hipStream_t s2, hipEvent_t e0, hipEvent_t e1) {
            Batch<PK> bb = b;
            void* a2[] = {&bb};
            if (e0)
                (void)hipExtLaunchKernel(k, grid, block, a2, sh, s2, e0, e1, 0);
            else
                (void)hipLaunchKernel(k, grid, block, a2, sh, s2);
        });
    return e;
}

template <class KS, class KB, class... A>
void batch_record_launch(KS ks, KB kb, const LaunchBytes& bytes, dim3 grid, dim3 block, size_t shmem, A&&... a) {
    using PK = typename PackOf<KS>::type;
    const PK pk = PackOf<KS>::as::make(static_cast<A&&>(a)...);
    BatchRec r;
    r.kernel = reinterpret_cast<const void*>(ks);
    r.batch_kernel = reinterpret_cast<const void*>(kb);
    r.grid = grid;
    r.block = block;
    r.shmem = shmem;
    r.bytes = bytes;
    r.pack.resize(sizeof(PK));
    std::memcpy(r.pack.data(), &pk, sizeof(PK));
    r.launch = &launch_batch_pack<PK>;
    batch_record(std::move(r));
}

}  // namespace ehh

#define EHH_EXPAND(...) __VA_ARGS__

// NAME<TARGS>(args) as one launch, or recorded for a batch (see above)
#define EHH_LAUNCHK(BYTES, NAME, TARGS, GRID, BLOCK, SHMEM, STREAM, ...)                                          \
    do {                                                                                                         \
        if (::ehh::batch_recording()) {                                                                          \
            using ehh_pk_ = typename ::ehh::PackOf<decltype(&NAME<EHH_EXPAND TARGS>)>::type;                     \
            ::ehh::batch_record_launch(&NAME<EHH_EXPAND TARGS>, &NAME##_batch<ehh_pk_, EHH_EXPAND TARGS>,        \
                                       (BYTES), dim3(GRID), dim3(BLOCK), (size_t)(SHMEM), __VA_ARGS__);         \
        } else {                                                                                                 \
            EHH_LAUNCH_B((BYTES), (NAME<EHH_EXPAND TARGS>), GRID, BLOCK, SHMEM, STREAM, __VA_ARGS__);            \
        }                                                                                                        \
    } while (0)
