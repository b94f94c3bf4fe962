// Host-only driver for the serving session's admission policy (scheduler.h):
// reads commands on stdin, prints what the scheduler does.  Used by
// test_scheduler_cpu.py.
//   arena CAP SLOTS BYPASS      new scheduler
//   push TICKET BYTES           queue a request
//   admit                       print "admit TICKET SLOT OFFSET" per admitted request
//   finish SLOT                 the request in SLOT is done
//   state                       print "state RUNNING WAITING USED LARGEST_FREE"
//   alloc BYTES / release OFF   raw arena operations on a separate arena of the same size
#include <iostream>
#include <memory>
#include <string>

#include "scheduler.h"

int main() {
    std::unique_ptr<ssr::serve::Scheduler> s;
    std::unique_ptr<ssr::serve::Arena> a;
    std::string cmd;
    while (std::cin >> cmd) {
        if (cmd == "arena") {
            long long cap;
            int slots, bypass;
            std::cin >> cap >> slots >> bypass;
            s.reset(new ssr::serve::Scheduler(cap, slots, bypass));
            a.reset(new ssr::serve::Arena(cap));
        } else if (cmd == "push") {
            unsigned long long t;
            long long b;
            std::cin >> t >> b;
            s->push(t, b);
        } else if (cmd == "admit") {
            for (const auto& ad : s->admit())
                std::cout << "admit " << ad.ticket << " " << ad.slot << " " << ad.offset << "\n";
        } else if (cmd == "finish") {
            int slot;
            std::cin >> slot;
            s->finish(slot);
        } else if (cmd == "state") {
            std::cout << "state " << s->running() << " " << s->waiting() << " " << s->arena().used()
                      << " " << s->arena().largest_free() << "\n";
        } else if (cmd == "alloc") {
            long long b;
            std::cin >> b;
            std::cout << "alloc " << a->alloc(b) << "\n";
        } else if (cmd == "release") {
            long long off;
            std::cin >> off;
            a->release(off);
            std::cout << "free " << a->used() << " " << a->largest_free() << "\n";
        }
    }
    return 0;
}
