// Command-line driver of the server's host-side admission pieces for the CPU
// tests: reads commands on stdin, prints results on stdout.
//   init BYTES
//   alloc ID BYTES      -> "ok OFFSET USED" | "fail USED"
//   free ID             -> "freed USED"
//   admit MAXBYPASS FREE N NEED_1 .. NEED_N B_1 .. B_N
//                       -> "admitted I ...  | bypasses K | counters C_1 .. C_N"
#include <cstdio>
#include <iostream>
#include <map>
#include <string>
#include <vector>

#include "arena.hpp"

int main() {
    fgs::Arena a;
    std::map<long, std::pair<size_t, size_t>> live;  // id -> (offset, bytes)
    std::string cmd;
    while (std::cin >> cmd) {
        if (cmd == "init") {
            size_t n;
            std::cin >> n;
            a.init(n);
            live.clear();
            std::printf("init %zu\n", a.size());
        } else if (cmd == "alloc") {
            long id;
            size_t n, off = 0;
            std::cin >> id >> n;
            if (a.alloc(n, &off)) {
                live[id] = {off, n};
                std::printf("ok %zu %zu\n", off, a.used());
            } else {
                std::printf("fail %zu\n", a.used());
            }
        } else if (cmd == "free") {
            long id;
            std::cin >> id;
            auto it = live.find(id);
            if (it != live.end()) {
                a.release(it->second.first, it->second.second);
                live.erase(it);
            }
            std::printf("freed %zu\n", a.used());
        } else if (cmd == "admit") {
            int maxb, n;
            long long freeb;
            std::cin >> maxb >> freeb >> n;
            std::vector<long long> need(n);
            std::vector<int> counters(n);
            for (auto &x : need) std::cin >> x;
            for (auto &x : counters) std::cin >> x;
            std::vector<int> idx(n);
            for (int i = 0; i < n; ++i) idx[i] = i;
            std::vector<int> admitted;
            auto try_admit = [&](int i) {
                if (need[i] > freeb) return false;
                freeb -= need[i];
                admitted.push_back(i);
                return true;
            };
            auto bypassed = [&](int i) -> int & { return counters[i]; };
            int64_t byp = 0;
            fgs::admit_fifo_bounded_bypass(idx, maxb, try_admit, bypassed, &byp);
            std::printf("admitted");
            for (int i : admitted) std::printf(" %d", i);
            std::printf(" | bypasses %lld | counters", (long long)byp);
            for (int c : counters) std::printf(" %d", c);
            std::printf("\n");
        }
    }
    return 0;
}
