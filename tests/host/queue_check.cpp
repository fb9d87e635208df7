// Host check of the batched work queue's ticket order and dependencies
// (queue_plan.h), with no GPU: random task lists, rounds built as the library
// builds them (no two batches of one plan, or with overlapping outputs, in a
// round; overlapping outputs in later rounds), then
//   1. every dependency names a counter whose tickets all come earlier;
//   2. a simulation of blocks that take tickets in order, each waiting on its
//      dependencies and finishing after a random time, always completes
//      (no wait on a later ticket can stall it), over many random timings;
//   3. in every simulated run: per batch, A finishes before any B ticket
//      starts, B before C, C before the finalize; a batch on a plan starts
//      pass A only after the previous batch on that plan finished pass C, and
//      pass C only after that batch's finalize; overlapping outputs are
//      written in round order; finalizes run one at a time in ticket order.
// Exit status 0 and "OK" when every check passes.
#include <cstdio>
#include <cstdlib>
#include <random>
#include <vector>

#include "queue_plan.h"

using kx::QBatchDesc;
using kx::QTicketDesc;

static int fails = 0;
#define CHECK(c, ...)                   \
  do {                                  \
    if (!(c)) {                         \
      std::printf("FAIL: " __VA_ARGS__); \
      std::printf("\n");                \
      ++fails;                          \
    }                                   \
  } while (0)

struct Task {
  int plan, n_b, nt;
  int out;  // output id: tasks with the same out write the same Vx range
};

// Batches in rounds, greedily in task order (as the library's schedule).
static std::vector<std::vector<QBatchDesc>> make_rounds(const std::vector<Task>& tasks, std::mt19937& rng) {
  struct Placed {
    QBatchDesc b;
    size_t round;
  };
  std::vector<Placed> placed;
  std::vector<std::vector<QBatchDesc>> rounds;
  std::uniform_int_distribution<int> cnt(1, 6);
  for (const Task& t : tasks) {
    for (int n0 = 0; n0 < t.n_b; n0 += t.nt) {
      const int cur = std::min(t.nt, t.n_b - n0);
      QBatchDesc b{t.plan, cnt(rng), cnt(rng), cnt(rng), (int)(rng() % 2),
                   (uintptr_t)(t.out * 1000 + n0), (uintptr_t)(t.out * 1000 + n0 + cur)};
      size_t r = 0;
      for (const Placed& q : placed)
        if (b.lo < q.b.hi && q.b.lo < b.hi) r = std::max(r, q.round + 1);
      for (;; ++r) {
        bool ok = true;
        for (const Placed& q : placed)
          if (q.round == r && q.b.plan == b.plan) ok = false;
        if (ok) break;
      }
      if (r >= rounds.size()) rounds.resize(r + 1);
      rounds[r].push_back(b);
      placed.push_back(Placed{b, r});
    }
  }
  return rounds;
}

int main() {
  std::mt19937 rng(1234);
  for (int trial = 0; trial < 300; ++trial) {
    const int ntask = 1 + (int)(rng() % 12), nplan = 1 + (int)(rng() % 5), nout = 1 + (int)(rng() % 6);
    std::vector<Task> tasks;
    for (int i = 0; i < ntask; ++i) {
      const int n_b = 1 + (int)(rng() % 20);
      tasks.push_back(Task{(int)(rng() % nplan), n_b, 1 + (int)(rng() % n_b), (int)(rng() % nout)});
    }
    const auto rounds = make_rounds(tasks, rng);
    std::vector<QBatchDesc> bs;
    std::vector<int> round_of;
    for (size_t r = 0; r < rounds.size(); ++r)
      for (const auto& b : rounds[r]) {
        bs.push_back(b);
        round_of.push_back((int)r);
      }
    const std::vector<QTicketDesc> tk = kx::queue_tickets(rounds);
    const int nctr = 4 * (int)bs.size();
    // tickets per counter and the last ticket index of each counter
    std::vector<int> per(nctr, 0), last(nctr, -1);
    for (size_t i = 0; i < tk.size(); ++i) {
      ++per[tk[i].done];
      last[tk[i].done] = (int)i;
    }
    for (int c = 0; c < nctr; ++c) {
      const QBatchDesc& b = bs[c / 4];
      const int want = c % 4 == 0 ? b.nA : c % 4 == 1 ? b.nB : c % 4 == 2 ? b.nC : b.fin;
      CHECK(per[c] == want, "trial %d: counter %d has %d tickets, %d expected", trial, c, per[c], want);
    }
    // 1. dependencies point to earlier tickets and to their full counts
    for (size_t i = 0; i < tk.size(); ++i)
      for (int k = 0; k < 3; ++k) {
        const int d = tk[i].dep[k];
        if (d < 0) continue;
        CHECK(d < nctr && last[d] >= 0 && last[d] < (int)i, "trial %d: ticket %zu waits on a later counter %d",
              trial, i, d);
        CHECK(tk[i].need[k] == per[d], "trial %d: ticket %zu needs %d of %d", trial, i, tk[i].need[k], per[d]);
      }
    // 2./3. simulated runs
    for (int run = 0; run < 20; ++run) {
      const int nblocks = 1 + (int)(rng() % 8);
      std::vector<int> ctr(nctr, 0);
      std::vector<long> start(tk.size(), -1), finish(tk.size(), -1);
      std::vector<int> held(nblocks, -1);
      std::vector<long> busy_until(nblocks, 0);
      size_t next = 0, done = 0;
      long now = 0;
      while (done < tk.size() && now < 10000000) {
        for (int bl = 0; bl < nblocks; ++bl) {
          if (held[bl] >= 0 && start[held[bl]] >= 0 && busy_until[bl] <= now) {  // finishes
            finish[held[bl]] = now;
            ++ctr[tk[held[bl]].done];
            ++done;
            held[bl] = -1;
          }
          if (held[bl] < 0 && next < tk.size()) held[bl] = (int)next++;  // takes the next ticket
          if (held[bl] >= 0 && start[held[bl]] < 0) {  // waiting: starts once its dependencies are met
            const QTicketDesc& t = tk[held[bl]];
            bool ok = true;
            for (int k = 0; k < 3; ++k)
              if (t.dep[k] >= 0 && ctr[t.dep[k]] < t.need[k]) ok = false;
            if (ok) {
              start[held[bl]] = now;
              busy_until[bl] = now + 1 + (long)(rng() % 7);
            }
          }
        }
        ++now;
      }
      CHECK(done == tk.size(), "trial %d run %d: stalled with %zu of %zu tickets done", trial, run, done, tk.size());
      if (done != tk.size()) continue;
      // per-pass first start / last finish of every batch
      const int nb = (int)bs.size();
      std::vector<long> s0(4 * nb, 1L << 60), f1(4 * nb, -1);
      for (size_t i = 0; i < tk.size(); ++i) {
        const int c = tk[i].done;
        s0[c] = std::min(s0[c], start[i]);
        f1[c] = std::max(f1[c], finish[i]);
      }
      for (int b = 0; b < nb; ++b) {
        CHECK(f1[4 * b] <= s0[4 * b + 1], "trial %d: batch %d pass B before A done", trial, b);
        CHECK(f1[4 * b + 1] <= s0[4 * b + 2], "trial %d: batch %d pass C before B done", trial, b);
        if (bs[b].fin) CHECK(f1[4 * b + 2] <= s0[4 * b + 3], "trial %d: batch %d finalize before C", trial, b);
        for (int a = 0; a < b; ++a) {
          if (round_of[a] >= round_of[b]) continue;
          if (bs[a].plan == bs[b].plan) {
            CHECK(f1[4 * a + 2] <= s0[4 * b], "trial %d: batch %d reuses a workspace before %d read it", trial, b, a);
            if (bs[a].fin)
              CHECK(f1[4 * a + 3] <= s0[4 * b + 2], "trial %d: batch %d overwrites partials of %d", trial, b, a);
          }
          if (bs[a].lo < bs[b].hi && bs[b].lo < bs[a].hi)
            CHECK(f1[4 * a + 2] <= s0[4 * b + 2], "trial %d: overlapping outputs %d, %d out of order", trial, a, b);
        }
      }
      // finalizes one at a time, in ticket order
      long prev_f = -1;
      for (size_t i = 0; i < tk.size(); ++i) {
        if (tk[i].pass != 3) continue;
        CHECK(start[i] >= prev_f, "trial %d: finalize %zu started before the previous one finished", trial, i);
        prev_f = finish[i];
      }
    }
  }
  if (fails) {
    std::printf("%d failures\n", fails);
    return 1;
  }
  std::printf("OK\n");
  return 0;
}
