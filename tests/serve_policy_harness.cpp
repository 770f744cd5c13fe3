// CPU harness for the serving loop's admission / batching policy
// (paper_2602_23067_amd/csrc/serve_policy.h): randomized arrivals and
// completions, checking the invariants the serving loop relies on.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "serve_policy.h"

using gcm::PolicyConfig;
using gcm::PolicyReq;
using gcm::ServePolicy;

#define CHECK(c)                                                             \
    do {                                                                     \
        if (!(c)) {                                                          \
            std::fprintf(stderr, "check failed line %d: %s\n", __LINE__, #c); \
            return 1;                                                        \
        }                                                                    \
    } while (0)

int main()
{
    for (unsigned seed = 1; seed <= 200; ++seed) {
        std::mt19937_64 rng(seed);
        PolicyConfig c;
        c.budget = 1000 + rng() % 100000;
        c.max_batch_reqs = 1 + rng() % 32;
        c.max_batch_bytes = 1 + rng() % 20000;
        c.max_queue = 1 + rng() % 500;
        ServePolicy p(c);
        uint64_t next = 1, expect_admit = 1, expect_batch = 1;
        std::vector<PolicyReq> running;
        uint64_t held = 0;
        for (int step = 0; step < 2000; ++step) {
            const int action = (int)(rng() % 4);
            if (action == 0) {  // arrival
                PolicyReq r{next, rng() % (c.budget + c.budget / 8 + 1), rng() % 30000};
                const int o = p.offer(r);
                if (r.need > c.budget) {
                    CHECK(o == ServePolicy::kTooLarge);
                } else if (o == ServePolicy::kAccepted) {
                    ++next;
                } else {
                    CHECK(o == ServePolicy::kQueueFull);
                    CHECK(p.pending() + p.ready() >= c.max_queue);
                }
            } else if (action == 1) {  // admission, strictly in arrival order
                std::vector<uint64_t> ids;
                p.admit(&ids);
                for (uint64_t id : ids)
                    CHECK(id == expect_admit++);
                CHECK(p.admitted_bytes() <= c.budget);
            } else if (action == 2) {  // batch formation
                std::vector<PolicyReq> b;
                if (p.next_batch(&b)) {
                    CHECK(b.size() <= c.max_batch_reqs);
                    uint64_t bytes = 0;
                    for (const PolicyReq &r : b) {
                        CHECK(r.id == expect_batch++);
                        bytes += r.payload;
                    }
                    CHECK(b.size() == 1 || bytes <= c.max_batch_bytes);
                    for (const PolicyReq &r : b) {
                        running.push_back(r);
                        held += r.need;
                    }
                }
            } else if (!running.empty() && rng() % 8) {  // completion of a random running request
                const size_t k = rng() % running.size();
                held -= running[k].need;
                // the stream slot that ran it keeps part of its scratch: bytes
                // move from the request's admission to the loop's slack
                const uint64_t keep = rng() % (running[k].need + 1);
                p.complete(running[k].need);
                p.set_slack(p.slack() + keep);
                running.erase(running.begin() + (long)k);
            } else {  // the loop frees idle slot memory
                p.set_slack(rng() % 2 ? 0 : p.slack() / 2);
            }
            CHECK(p.admitted_bytes() <= c.budget);
            CHECK(p.admitted_bytes() + p.slack() <= c.budget);
            CHECK(p.high_water() <= c.budget);
            CHECK(held <= p.admitted_bytes());
        }
        // drain: everything eventually admitted and batched once running work completes
        for (const PolicyReq &r : running)
            p.complete(r.need);
        running.clear();
        std::vector<PolicyReq> b;
        for (int guard = 0; guard < 100000 && (p.pending() || p.ready()); ++guard) {
            if (!p.admit() && p.ready() == 0)
                p.set_slack(0);  // nothing runs and the head does not fit: free idle slot memory
            while (p.next_batch(&b))
                for (const PolicyReq &r : b)
                    p.complete(r.need);
        }
        CHECK(p.pending() == 0 && p.ready() == 0 && p.admitted_bytes() == 0);
    }
    std::printf("serve policy: OK\n");
    return 0;
}
