// Admission control of the serving session: the device-memory arena that
// request workspaces are carved from, and the queue that admits waiting
// requests as slots and memory free up.  Plain C++ (no HIP), so the policy
// runs and is tested on the host alone.
#pragma once

#include <stdint.h>

#include <deque>
#include <iterator>
#include <map>
#include <vector>

namespace ssr {
namespace serve {

// First-fit allocator of byte ranges in [0, capacity), aligned to `align`,
// with neighbouring free ranges merged on release.
class Arena {
 public:
    explicit Arena(int64_t capacity = 0, int64_t align = 256) : cap_(capacity), align_(align) {
        if (cap_ > 0) free_[0] = cap_;
    }
    int64_t capacity() const { return cap_; }
    int64_t used() const { return used_bytes_; }
    int64_t round(int64_t n) const { return (n + align_ - 1) / align_ * align_; }

    // Offset of a new range of `size` bytes, or -1 if no free range holds it.
    int64_t alloc(int64_t size) {
        size = round(size > 0 ? size : 1);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second < size) continue;
            const int64_t off = it->first, rest = it->second - size;
            free_.erase(it);
            if (rest > 0) free_[off + size] = rest;
            used_[off] = size;
            used_bytes_ += size;
            return off;
        }
        return -1;
    }

    // Release the range that starts at `off` (unknown offsets are ignored).
    void release(int64_t off) {
        auto u = used_.find(off);
        if (u == used_.end()) return;
        int64_t start = off, size = u->second;
        used_bytes_ -= size;
        used_.erase(u);
        auto next = free_.lower_bound(start);
        if (next != free_.end() && start + size == next->first) {
            size += next->second;
            next = free_.erase(next);
        }
        if (next != free_.begin()) {
            auto prev = std::prev(next);
            if (prev->first + prev->second == start) {
                start = prev->first;
                size += prev->second;
                free_.erase(prev);
            }
        }
        free_[start] = size;
    }

    // The largest range alloc() could return now.
    int64_t largest_free() const {
        int64_t m = 0;
        for (const auto& f : free_) m = f.second > m ? f.second : m;
        return m;
    }

 private:
    int64_t cap_, align_;
    int64_t used_bytes_ = 0;
    std::map<int64_t, int64_t> free_;   // offset -> size
    std::map<int64_t, int64_t> used_;   // offset -> size
};

struct Admitted {
    uint64_t ticket;
    int slot;
    int64_t offset;   // of the request's workspace in the arena
};

// Waiting requests in arrival order, admitted when a slot is free and the
// arena holds their workspace.  A request that does not fit may be overtaken
// by later, smaller ones, but only max_bypass times: after that nothing is
// admitted ahead of it, so no request waits forever while others keep
// arriving.
class Scheduler {
 public:
    Scheduler(int64_t arena_bytes, int slots, int max_bypass)
        : arena_(arena_bytes), max_bypass_(max_bypass < 0 ? 0 : max_bypass) {
        for (int s = slots - 1; s >= 0; --s) free_slots_.push_back(s);
        running_.assign(slots, Running{});
    }

    const Arena& arena() const { return arena_; }
    int64_t workspace(int64_t bytes) const { return arena_.round(bytes); }
    bool fits_ever(int64_t bytes) const { return arena_.round(bytes) <= arena_.capacity(); }

    void push(uint64_t ticket, int64_t bytes) { wait_.push_back(Waiting{ticket, bytes, 0}); }

    // Admit what can start now, oldest first.
    std::vector<Admitted> admit() {
        std::vector<Admitted> out;
        bool blocked = false;   // an older request is waiting for memory
        for (auto it = wait_.begin(); it != wait_.end() && !free_slots_.empty();) {
            if (blocked && wait_.front().bypassed >= max_bypass_) break;
            const int64_t off = arena_.alloc(it->bytes);
            if (off < 0) {
                blocked = true;
                ++it;
                continue;
            }
            const int slot = free_slots_.back();
            free_slots_.pop_back();
            running_[slot] = Running{true, it->ticket, off};
            out.push_back(Admitted{it->ticket, slot, off});
            if (blocked) ++wait_.front().bypassed;
            it = wait_.erase(it);
        }
        return out;
    }

    // The request in `slot` has finished: its slot and workspace are free.
    void finish(int slot) {
        if (slot < 0 || slot >= static_cast<int>(running_.size()) || !running_[slot].busy) return;
        arena_.release(running_[slot].offset);
        running_[slot] = Running{};
        free_slots_.push_back(slot);
    }

    // Drop every waiting request; returns their tickets.
    std::vector<uint64_t> drop_waiting() {
        std::vector<uint64_t> t;
        for (const auto& w : wait_) t.push_back(w.ticket);
        wait_.clear();
        return t;
    }

    int running() const { return static_cast<int>(running_.size() - free_slots_.size()); }
    int waiting() const { return static_cast<int>(wait_.size()); }
    bool idle() const { return wait_.empty() && running() == 0; }
    uint64_t ticket_in(int slot) const { return running_[slot].ticket; }
    bool busy(int slot) const { return running_[slot].busy; }
    int slots() const { return static_cast<int>(running_.size()); }

 private:
    struct Waiting {
        uint64_t ticket;
        int64_t bytes;
        int bypassed;
    };
    struct Running {
        bool busy = false;
        uint64_t ticket = 0;
        int64_t offset = 0;
    };
    Arena arena_;
    int max_bypass_;
    std::deque<Waiting> wait_;
    std::vector<int> free_slots_;
    std::vector<Running> running_;
};

}  // namespace serve
}  // namespace ssr
