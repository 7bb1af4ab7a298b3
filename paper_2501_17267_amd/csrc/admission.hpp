// admission.hpp -- the anneal server's admission policy, free of device
// calls so that it can be tested on the host with a scripted clock.
//
// Queued requests are considered in arrival order.  A request is admitted
// when the active limit, the memory budget and (for lattices whose spins
// live in a workspace) a free workspace slot allow it.  A request that does
// not fit is passed over, so that smaller requests behind it are not held
// up by it -- but only while it is younger than skip_age seconds: once the
// oldest such request has waited that long, nothing queued behind it is
// admitted until it fits, so it cannot starve.
#pragma once

#include <cstdint>
#include <deque>
#include <vector>

namespace sg {

struct AdmitEntry {
    uint64_t id;
    int64_t footprint;   // bytes of request state charged to the budget
    bool needs_ws;       // takes one of the large-lattice workspace slots
    double t_queued;     // when it entered the queue (server clock)
};

struct AdmitCapacity {
    int64_t active, max_active;
    int64_t mem_in_use, budget;
    int64_t ws_free;
};

// Removes from q the entries to admit now (returned in admission order)
// and those for which dropped(id) is true (cancelled while queued), and
// charges the admitted ones to cap.
template <class Dropped>
std::vector<AdmitEntry> admit_pick(std::deque<AdmitEntry> &q, AdmitCapacity &cap, double now, double skip_age,
                                   Dropped dropped)
{
    std::vector<AdmitEntry> out;
    std::deque<AdmitEntry> keep;
    bool blocked = false;   // an old request is waiting: admit nothing after it
    for (const AdmitEntry &e : q) {
        if (dropped(e.id)) continue;
        if (blocked || cap.active >= cap.max_active) {
            keep.push_back(e);
            continue;
        }
        const bool fits = cap.mem_in_use + e.footprint <= cap.budget && (!e.needs_ws || cap.ws_free > 0);
        if (fits) {
            cap.mem_in_use += e.footprint;
            cap.active += 1;
            if (e.needs_ws) cap.ws_free -= 1;
            out.push_back(e);
        } else {
            keep.push_back(e);
            if (now - e.t_queued >= skip_age) blocked = true;
        }
    }
    q.swap(keep);
    return out;
}

}  // namespace sg
