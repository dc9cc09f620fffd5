// Host test of the serving scheduler core (paper_2501_00675_amd/csrc/serve_sched.h)
// with a fake executor: requests of random footprint, plan and stage count
// are submitted, admitted, stepped and retired (or cancelled while queued);
// every step checks the invariants the server relies on.  Exit status 0 when
// every check holds.  Built and run by tests/test_sched_host.py.
#include <cstdio>
#include <cstdlib>
#include <deque>
#include <map>
#include <random>
#include <vector>

#include "serve_sched.h"

using namespace cosdag;

struct FakeReq {
    int id = 0;
    uint64_t footprint = 0, arena_off = 0;
    int slot = -1;
    bool fused = false;
    int section = 0;  // 0 / 2: whole-graph work, 1 / 3: streamed work (rational / lookup factors)
    int next_stage = 0, n_stages = 0;
    int bypassed = 0;
    int admitted_step = -1, done_step = -1;
    int last_stage_step = -1;
    bool cancelled = false;
};

static int failures = 0;
#define CHECK(cond, ...)                                  \
    do {                                                  \
        if (!(cond)) {                                    \
            std::fprintf(stderr, "FAIL %s:%d: ", __FILE__, __LINE__); \
            std::fprintf(stderr, __VA_ARGS__);            \
            std::fprintf(stderr, "\n");                   \
            if (++failures > 20)                          \
                std::exit(1);                             \
        }                                                 \
    } while (0)

static void arena_unit() {
    Arena a(4096);
    uint64_t o1, o2, o3, o4;
    CHECK(a.alloc(100, &o1) && o1 == 0, "first fit at 0");
    CHECK(a.alloc(256, &o2) && o2 == 256, "granule rounding");
    CHECK(a.alloc(1000, &o3) && o3 == 512, "third block");
    CHECK(!a.alloc(4096, &o4), "too large");
    a.release(o2, 256);
    CHECK(a.alloc(200, &o4) && o4 == 256, "reuse the freed hole first");
    a.release(o1, 100);
    a.release(o4, 200);
    a.release(o3, 1000);
    CHECK(a.used() == 0 && a.free_blocks().size() == 1 && a.free_blocks().front().second == 4096,
          "everything coalesces back into one block");
}

static void simulate(uint32_t seed, int n_req, int max_slots, uint64_t budget) {
    std::mt19937_64 rng(seed);
    std::vector<FakeReq> reqs(n_req);
    std::deque<FakeReq *> queue;
    std::vector<FakeReq *> slots(max_slots, nullptr);
    Arena arena(budget);
    int submitted = 0, done = 0, cancelled = 0;
    for (int step = 0; step < 100000 && done + cancelled < n_req; ++step) {
        // a few arrivals per step
        for (int k = static_cast<int>(rng() % 4); k > 0 && submitted < n_req; --k) {
            FakeReq &r = reqs[submitted];
            r.id = submitted++;
            r.fused = rng() % 3 == 0;
            r.section = (r.fused ? 0 : 1) + (rng() % 4 == 0 ? 2 : 0);
            r.footprint = r.fused ? 0 : 256 + rng() % (budget / 2);
            r.n_stages = r.fused ? 1 : 3 + static_cast<int>(rng() % 18);
            queue.push_back(&r);
        }
        // occasionally cancel a queued request
        if (!queue.empty() && rng() % 17 == 0) {
            auto it = queue.begin() + static_cast<long>(rng() % queue.size());
            (*it)->cancelled = true;
            queue.erase(it);
            ++cancelled;
        }
        const std::deque<FakeReq *> before = queue;
        const auto admitted = admit(queue, slots, arena);
        for (FakeReq *r : admitted)
            r->admitted_step = step;
        // admission order and skipping: a queued request passed over must not have fitted
        size_t ai = 0;
        for (FakeReq *q : before) {
            if (ai < admitted.size() && admitted[ai] == q) {
                ++ai;
                continue;
            }
            const bool still_queued = std::find(queue.begin(), queue.end(), q) != queue.end();
            CHECK(still_queued, "request %d vanished from the queue", q->id);
        }
        CHECK(ai == admitted.size(), "admitted requests are taken in queue order");
        // arena and slot invariants
        CHECK(arena.used() <= budget, "arena over budget");
        std::map<uint64_t, uint64_t> live;
        int active = 0;
        for (int sl = 0; sl < max_slots; ++sl) {
            FakeReq *r = slots[sl];
            if (!r)
                continue;
            ++active;
            CHECK(r->slot == sl, "slot index");
            if (r->footprint)
                live[r->arena_off] = Arena::granules(r->footprint);
        }
        uint64_t end = 0, sum = 0;
        for (auto &kv : live) {
            CHECK(kv.first >= end, "workspaces overlap at %llu", static_cast<unsigned long long>(kv.first));
            end = kv.first + kv.second;
            sum += kv.second;
        }
        CHECK(end <= budget && sum == arena.used(), "arena accounting");
        // a request not admitted while a slot was free must not fit in the largest free block,
        // unless an earlier request that does not fit has been passed over kMaxBypass times
        if (active < max_slots) {
            uint64_t largest = 0;
            for (auto &b : arena.free_blocks())
                largest = std::max(largest, b.second);
            for (FakeReq *q : queue) {
                const bool fits = q->footprint == 0 || Arena::granules(q->footprint) <= largest;
                if (!fits && q->bypassed >= kMaxBypass)
                    break;
                CHECK(!fits, "request %d fits but was not admitted", q->id);
            }
        }
        for (FakeReq *q : queue)
            CHECK(q->bypassed <= kMaxBypass, "request %d passed over %d times", q->id, q->bypassed);
        // compose and run one step
        if (!any_stage_left(slots))
            continue;
        int out_of_order = 0, last_section = 0;
        std::vector<FakeReq *> finishing;
        const int n = compose_step(slots, 4, [&](int section, FakeReq *r) {
            out_of_order += section < last_section;
            last_section = section;
            CHECK(r->last_stage_step < step, "two stages of request %d in one step", r->id);
            CHECK(r->section == section, "section of request %d", r->id);
            r->last_stage_step = step;
            if (r->next_stage + 1 == r->n_stages)
                finishing.push_back(r);
        });
        CHECK(n > 0 && out_of_order == 0, "entries come grouped by section, in section order");
        // the fake executor completes the step: retire finished requests
        for (FakeReq *r : finishing) {
            CHECK(r->next_stage == r->n_stages, "request %d retired early", r->id);
            CHECK(step - r->admitted_step + 1 == r->n_stages, "request %d took %d steps for %d stages", r->id,
                  step - r->admitted_step + 1, r->n_stages);
            r->done_step = step;
            if (r->footprint)
                arena.release(r->arena_off, r->footprint);
            slots[r->slot] = nullptr;
            ++done;
        }
    }
    CHECK(done + cancelled == n_req, "only %d of %d requests ended", done + cancelled, n_req);
    CHECK(arena.used() == 0 && arena.free_blocks().size() == 1, "arena not fully coalesced at the end");
    for (FakeReq &r : reqs)
        CHECK(r.cancelled || r.done_step >= 0, "request %d never finished", r.id);
    // counted independently of admit(): later requests admitted before each request
    for (FakeReq &r : reqs) {
        if (r.cancelled)
            continue;
        int ahead = 0;
        for (FakeReq &q : reqs)
            ahead += q.id > r.id && !q.cancelled && q.admitted_step < r.admitted_step;
        CHECK(ahead <= kMaxBypass && ahead == r.bypassed, "request %d: %d later requests went first (count %d)",
              r.id, ahead, r.bypassed);
    }
}

// A large request queued behind a steady stream of small ones that each live two
// steps: without a bound the arena never has room for it; with it, the small ones
// stop after kMaxBypass admissions ahead of it, drain, and it is admitted.
static void bypass_unit() {
    const uint64_t G = Arena::kGranule;
    Arena arena(10 * G);
    std::vector<FakeReq *> slots(4, nullptr);
    std::deque<FakeReq *> queue;
    std::vector<FakeReq> reqs(400);
    FakeReq &big = reqs[0];
    big.id = 0;
    big.footprint = 9 * G;
    std::vector<std::pair<FakeReq *, int>> live;  // (request, retire step)
    FakeReq first;
    first.footprint = 2 * G;
    std::deque<FakeReq *> q0{&first};
    admit(q0, slots, arena);
    live.push_back({&first, 1});
    queue.push_back(&big);
    int next = 1, big_step = -1;
    for (int step = 0; step < 200 && big_step < 0; ++step) {
        if (next < static_cast<int>(reqs.size())) {  // one small arrival per step
            reqs[next].id = next;
            reqs[next].footprint = G;
            queue.push_back(&reqs[next++]);
        }
        for (FakeReq *r : admit(queue, slots, arena)) {
            if (r == &big)
                big_step = step;
            else
                live.push_back({r, step + 2});
        }
        for (auto it = live.begin(); it != live.end();) {
            if (it->second == step) {
                arena.release(it->first->arena_off, it->first->footprint);
                slots[it->first->slot] = nullptr;
                it = live.erase(it);
            } else {
                ++it;
            }
        }
    }
    CHECK(big_step >= 0, "the large request was never admitted");
    CHECK(big.bypassed == kMaxBypass, "the large request was passed over %d times", big.bypassed);
}

int main() {
    arena_unit();
    bypass_unit();
    simulate(1, 400, 8, 1 << 20);
    simulate(2, 400, 64, 1 << 22);
    simulate(3, 300, 1, 1 << 16);   // one slot: strictly one request at a time
    simulate(4, 500, 512, 1 << 18); // budget-bound: many slots, little memory
    if (failures) {
        std::fprintf(stderr, "%d check(s) failed\n", failures);
        return 1;
    }
    std::printf("scheduler checks passed\n");
    return 0;
}
