// serve_policy.h -- admission and continuous-batching policy of the serving
// loop.  It holds no HIP state, so the same code runs inside the library and
// in a CPU-only test harness.
//
// Requests wait in arrival order.  A request is admitted when the bytes it
// needs on the device (its input, output and AAD, plus its share of a
// batch's descriptors, work list and tile partials) fit in what is left of
// the HBM budget after the serving loop's own retained scratch (`slack`:
// stream-slot memory not used by a running batch); admission never skips
// ahead of an earlier request, so no request starves.  Admitted requests are
// handed out in arrival order as batches of at most max_batch_reqs requests
// and about max_batch_bytes of payload (a single larger request forms a batch
// of its own).  Completing a request returns its bytes to the budget.
#pragma once
#include <cstdint>
#include <deque>
#include <vector>

namespace gcm {

struct PolicyConfig {
    uint64_t budget = 64ull << 30;
    uint32_t max_batch_reqs = 256;
    uint64_t max_batch_bytes = 256ull << 20;
    uint32_t max_queue = 1u << 16;
};

struct PolicyReq {
    uint64_t id;
    uint64_t need;     // device bytes held while admitted
    uint64_t payload;  // payload bytes (batch sizing)
};

class ServePolicy {
  public:
    enum Offer { kAccepted = 0, kTooLarge = -1, kQueueFull = -2 };

    explicit ServePolicy(PolicyConfig c = PolicyConfig()) : cfg_(c) {}

    int offer(const PolicyReq &r)
    {
        if (r.need > cfg_.budget)
            return kTooLarge;
        if (pending_.size() + ready_.size() >= cfg_.max_queue)
            return kQueueFull;
        pending_.push_back(r);
        return kAccepted;
    }

    // Admit from the head of the queue while the budget allows.
    size_t admit(std::vector<uint64_t> *admitted = nullptr)
    {
        size_t k = 0;
        while (!pending_.empty() && slack_ <= cfg_.budget && admitted_ <= cfg_.budget - slack_ &&
               pending_.front().need <= cfg_.budget - slack_ - admitted_) {
            admitted_ += pending_.front().need;
            if (admitted_ + slack_ > high_)
                high_ = admitted_ + slack_;
            if (admitted)
                admitted->push_back(pending_.front().id);
            ready_.push_back(pending_.front());
            pending_.pop_front();
            ++k;
        }
        return k;
    }

    // Next batch of admitted requests, in arrival order.
    bool next_batch(std::vector<PolicyReq> *out)
    {
        out->clear();
        uint64_t bytes = 0;
        while (!ready_.empty() && out->size() < cfg_.max_batch_reqs) {
            const PolicyReq &r = ready_.front();
            if (!out->empty() && bytes + r.payload > cfg_.max_batch_bytes)
                break;
            bytes += r.payload;
            out->push_back(r);
            ready_.pop_front();
        }
        return !out->empty();
    }

    void complete(uint64_t need) { admitted_ -= need; }

    // Device bytes the serving loop retains beyond what admitted requests
    // account for (counted against the budget).
    void set_slack(uint64_t bytes)
    {
        slack_ = bytes;
        if (admitted_ + slack_ > high_)
            high_ = admitted_ + slack_;
    }
    uint64_t slack() const { return slack_; }

    uint64_t admitted_bytes() const { return admitted_; }
    uint64_t high_water() const { return high_; }
    size_t pending() const { return pending_.size(); }
    size_t ready() const { return ready_.size(); }
    const PolicyConfig &config() const { return cfg_; }

  private:
    PolicyConfig cfg_;
    std::deque<PolicyReq> pending_, ready_;
    uint64_t admitted_ = 0, high_ = 0, slack_ = 0;
};

}  // namespace gcm
