// server_policy.h -- admission policy of the product server (host code only).
//
// Requests wait in arrival order.  A request is admitted when a launch slot
// is free and its workspace fits in the server's device-memory arena; small
// products (at most `batch_limit_bits`) are grouped, in arrival order, into
// one batched launch, large ones (and every product on a resident operand's
// kept transform) run on a slot of their own.  A later request
// may pass an earlier one that does not fit yet, but a request that has been
// passed `starve_after` times blocks all later ones until it is admitted.
#pragma once

#include <cstdint>
#include <deque>
#include <functional>
#include <iterator>
#include <map>
#include <vector>

namespace fpmul_srv {

// first-fit allocator over [0, size) with coalescing; granularity 256 bytes
class Arena {
public:
    explicit Arena(uint64_t size = 0) { reset(size); }
    void reset(uint64_t size)
    {
        free_.clear();
        size_ = size & ~255ull;
        if (size_) free_[0] = size_;
    }
    uint64_t size() const { return size_; }
    static uint64_t round(uint64_t bytes) { return (bytes + 255) & ~255ull; }
    bool alloc(uint64_t bytes, uint64_t &off)
    {
        bytes = round(bytes ? bytes : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < bytes) continue;
            off = it->first;
            const uint64_t rest = it->second - bytes;
            free_.erase(it);
            if (rest) free_[off + bytes] = rest;
            return true;
        }
        return false;
    }
    void release(uint64_t off, uint64_t bytes)
    {
        bytes = round(bytes ? bytes : 1);
        auto next = free_.lower_bound(off);
        if (next != free_.end() && next->first == off + bytes) {
            bytes += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == off) {
                prev->second += bytes;
                return;
            }
        }
        free_[off] = bytes;
    }
    uint64_t free_bytes() const
    {
        uint64_t s = 0;
        for (const auto &kv : free_) s += kv.second;
        return s;
    }
    uint64_t largest_free() const
    {
        uint64_t m = 0;
        for (const auto &kv : free_) m = kv.second > m ? kv.second : m;
        return m;
    }

private:
    std::map<uint64_t, uint64_t> free_;
    uint64_t size_ = 0;
};

struct Req {
    uint64_t ticket = 0;
    uint64_t la = 0, lb = 0;
    const uint64_t *a = nullptr, *b = nullptr;
    uint64_t *out = nullptr;
    uint32_t skipped = 0;
    // a request on a resident operand: A's forward transform of 2^res_log2n
    // bits is kept on the device (fa); it always runs alone, on the
    // workspace of that transform length
    const uint64_t *fa = nullptr;
    int res_log2n = 0;
};

struct Policy {
    uint64_t batch_limit_bits = 1ull << 20;   // products at or below go to batched launches
    uint32_t max_batch = 512;                 // requests per batched launch
    uint32_t starve_after = 64;               // passes before a waiting request blocks later ones
};

// device bytes a launch needs: single(lc) for one product of lc bits,
// batch(count, largest lc) for a batched launch
struct Footprint {
    std::function<uint64_t(uint64_t lc)> single;
    std::function<uint64_t(uint32_t count, uint64_t max_lc)> batch;
};

struct Plan {
    bool batch = false;
    std::vector<Req> reqs;
    uint64_t off = 0, bytes = 0;   // arena range
    uint64_t max_lc = 0;
};

inline uint64_t product_bits(const Req &r) { return r.la + r.lb - 1; }

// the length whose single-launch footprint holds the request
inline uint64_t launch_bits(const Req &r) { return r.fa ? (1ull << r.res_log2n) : product_bits(r); }

// Takes the next launch out of `pending` if one can be admitted now.
inline bool next_plan(std::deque<Req> &pending, Arena &arena, const Policy &P, const Footprint &F, Plan &out)
{
    const size_t n = pending.size();
    for (size_t idx = 0; idx < n; ++idx) {
        if (idx > 0 && pending[0].skipped >= P.starve_after) break;
        const Req &r = pending[idx];
        std::vector<size_t> group;
        uint64_t bytes = 0, max_lc = 0;
        bool batch = !r.fa && product_bits(r) <= P.batch_limit_bits;
        uint64_t off = 0;
        if (batch) {
            for (size_t j = idx; j < n && group.size() < P.max_batch; ++j) {
                const Req &q = pending[j];
                if (q.fa || product_bits(q) > P.batch_limit_bits) continue;
                group.push_back(j);
                max_lc = product_bits(q) > max_lc ? product_bits(q) : max_lc;
            }
            bytes = F.batch((uint32_t)group.size(), max_lc);
            if (!arena.alloc(bytes, off)) {
                group.assign(1, idx);
                max_lc = product_bits(r);
                bytes = F.batch(1, max_lc);
                if (!arena.alloc(bytes, off)) continue;
            }
        } else {
            group.assign(1, idx);
            max_lc = launch_bits(r);
            bytes = F.single(max_lc);
            if (!arena.alloc(bytes, off)) continue;
        }
        // admitted: every waiting request before the last admitted one is passed
        const size_t last = group.back();
        size_t g = 0;
        for (size_t j = 0; j < last; ++j) {
            if (g < group.size() && group[g] == j) {
                ++g;
                continue;
            }
            pending[j].skipped++;
        }
        out.batch = batch;
        out.reqs.clear();
        for (size_t j : group) out.reqs.push_back(pending[j]);
        out.off = off;
        out.bytes = bytes;
        out.max_lc = max_lc;
        for (auto it = group.rbegin(); it != group.rend(); ++it) pending.erase(pending.begin() + (long)*it);
        return true;
    }
    return false;
}

}  // namespace fpmul_srv
