// Host-side scheduling core of the serving runtime, free of device calls so
// that it can be exercised on its own: the workspace arena, admission of
// queued requests by slot and footprint, and the composition of a step from
// the active requests' next stages.  The server (server.cpp) drives it under
// its lock; a request type only needs the fields used here.
#pragma once

#include <algorithm>
#include <cstdint>
#include <deque>
#include <list>
#include <utility>
#include <vector>

namespace cosdag {

// First-fit allocator over [0, size) with coalescing, 256-byte granules.
class Arena {
  public:
    static constexpr uint64_t kGranule = 256;
    explicit Arena(uint64_t size) : size_(size) {
        if (size)
            free_.push_back({0, size});
    }
    static uint64_t granules(uint64_t n) { return (std::max<uint64_t>(n, 1) + kGranule - 1) / kGranule * kGranule; }
    bool alloc(uint64_t n, uint64_t *off) {
        n = granules(n);
        for (auto it = free_.begin(); it != free_.end(); ++it) {
            if (it->second >= n) {
                *off = it->first;
                it->first += n;
                it->second -= n;
                if (it->second == 0)
                    free_.erase(it);
                used_ += n;
                return true;
            }
        }
        return false;
    }
    void release(uint64_t off, uint64_t n) {
        n = granules(n);
        used_ -= n;
        auto it = free_.begin();
        while (it != free_.end() && it->first < off)
            ++it;
        it = free_.insert(it, {off, n});
        auto next = std::next(it);
        if (next != free_.end() && it->first + it->second == next->first) {
            it->second += next->second;
            free_.erase(next);
        }
        if (it != free_.begin()) {
            auto prev = std::prev(it);
            if (prev->first + prev->second == it->first) {
                prev->second += it->second;
                free_.erase(it);
            }
        }
    }
    uint64_t used() const { return used_; }
    uint64_t size() const { return size_; }
    const std::list<std::pair<uint64_t, uint64_t>> &free_blocks() const { return free_; }

  private:
    uint64_t size_;
    uint64_t used_ = 0;
    std::list<std::pair<uint64_t, uint64_t>> free_;  // (offset, bytes), sorted by offset
};

// How many later requests may be admitted ahead of a queued request whose
// workspace does not fit yet.
constexpr int kMaxBypass = 32;

// Admit queued requests in order while a slot is free: a request whose
// workspace (footprint bytes, 0 for none) does not fit in the arena now stays
// queued without blocking the ones behind it -- but only until max_bypass
// later requests have been admitted ahead of it (its bypassed count).  From
// then on admission stops at it until its workspace fits, which the
// completion of active requests guarantees (every footprint fits the whole
// arena), so no request waits without bound behind a stream of smaller ones.
// Admitted requests get a slot (the lowest free) and arena_off; returns them
// in admission order.  Req needs: footprint, arena_off, slot, bypassed.
template <class Req>
std::vector<Req *> admit(std::deque<Req *> &queue, std::vector<Req *> &slots, Arena &arena,
                         int max_bypass = kMaxBypass) {
    std::vector<Req *> admitted;
    std::vector<Req *> waiting;  // requests passed over in this call
    int free_slots = 0;
    for (Req *r : slots)
        free_slots += r == nullptr;
    for (auto it = queue.begin(); it != queue.end() && free_slots > 0;) {
        Req *r = *it;
        uint64_t off = 0;
        if (r->footprint && !arena.alloc(r->footprint, &off)) {
            if (r->bypassed >= max_bypass)
                break;  // its turn: nothing behind it goes first
            waiting.push_back(r);
            ++it;
            continue;
        }
        r->arena_off = off;
        r->slot = static_cast<int>(std::find(slots.begin(), slots.end(), nullptr) - slots.begin());
        slots[r->slot] = r;
        --free_slots;
        admitted.push_back(r);
        it = queue.erase(it);
        bool hold = false;
        for (Req *w : waiting)
            hold |= ++w->bypassed >= max_bypass;
        if (hold)
            break;
    }
    return admitted;
}

// Compose one step: every active request with a stage left contributes its
// next stage, grouped by section (0 .. n_sections-1, each run by its own
// kernel), each section in slot order; emit(section, request) is called for
// each in that order, and the request's next_stage advances.  Returns how
// many requests the step holds.  Req needs: section, next_stage, n_stages.
template <class Req, class Emit>
int compose_step(const std::vector<Req *> &slots, int n_sections, Emit emit) {
    int n = 0;
    for (int section = 0; section < n_sections; ++section)
        for (Req *r : slots) {
            if (!r || r->next_stage >= r->n_stages || r->section != section)
                continue;
            emit(section, r);
            ++r->next_stage;
            ++n;
        }
    return n;
}

// Whether some active request still has a stage to run.
template <class Req>
bool any_stage_left(const std::vector<Req *> &slots) {
    for (Req *r : slots)
        if (r && r->next_stage < r->n_stages)
            return true;
    return false;
}

}  // namespace cosdag
