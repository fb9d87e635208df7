// Ticket order and dependencies of the batched entry point's work queue
// (host-only, plain C++; the device side is kernels_queue.hip).
//
// Input: the batches of a task list in rounds (a round never holds two
// batches of one plan or two batches with overlapping Vx outputs), each with
// its plan, its Vx byte range and its ticket counts per pass.  Output: the
// tickets in order -- round by round, and within a round every batch's
// pass-A tickets, then pass B, pass C and the E_x finalizes -- each with the
// completion counter it increments (4 b + pass for batch b, pass 3 = the
// finalize) and up to three counters it waits on:
//   pass A  the previous batch on the same plan has finished pass C (the
//           plan's workspace is reused);
//   pass B  its own pass A;
//   pass C  its own pass B; the latest earlier batch with an overlapping Vx
//           range has finished pass C (outputs accumulate in task order); the
//           previous batch on the same plan has finalized (its E_x partials);
//   final   its own pass C; the previous finalize ticket (E_x accumulates in
//           a fixed order).
// Every dependency is on tickets that come earlier in the order.
#pragma once

#include <cstdint>
#include <vector>

namespace kx {

struct QBatchDesc {
  int plan;                 // plan identity (batches of one plan share a workspace)
  int nA, nB, nC, fin;      // tickets of passes A, B, C; 1 if the batch has a finalize
  uintptr_t lo, hi;         // Vx byte range [lo, hi)
};

struct QTicketDesc {
  int pass;                 // 0, 1, 2 = passes A, B, C; 3 = E_x finalize
  int batch;                // index in round order
  int vb, vg;               // virtual block and grid of the pass
  int done;                 // counter incremented on completion
  int dep[3], need[3];      // counters waited on (-1: none) and their targets
};

inline std::vector<QTicketDesc> queue_tickets(const std::vector<std::vector<QBatchDesc>>& rounds) {
  std::vector<QTicketDesc> out;
  std::vector<QBatchDesc> bs;  // all batches in round order
  int fin_prev = -1;
  for (const auto& round : rounds) {
    const size_t first = bs.size();
    for (const QBatchDesc& b : round) bs.push_back(b);
    auto prev_same_plan = [&](size_t bi) -> int {
      for (size_t j = first; j-- > 0;)
        if (bs[j].plan == bs[bi].plan) return (int)j;
      return -1;
    };
    auto prev_overlap = [&](size_t bi) -> int {
      for (size_t j = first; j-- > 0;)
        if (bs[bi].lo < bs[j].hi && bs[j].lo < bs[bi].hi) return (int)j;
      return -1;
    };
    for (int pass = 0; pass < 4; ++pass) {
      for (size_t bi = first; bi < bs.size(); ++bi) {
        const QBatchDesc& b = bs[bi];
        const int n = pass == 0 ? b.nA : pass == 1 ? b.nB : pass == 2 ? b.nC : b.fin;
        for (int v = 0; v < n; ++v) {
          QTicketDesc t{};
          t.pass = pass;
          t.batch = (int)bi;
          t.vb = v;
          t.vg = n;
          t.done = 4 * (int)bi + pass;
          for (int i = 0; i < 3; ++i) {
            t.dep[i] = -1;
            t.need[i] = 0;
          }
          if (pass == 0) {
            const int pp = prev_same_plan(bi);
            if (pp >= 0) {
              t.dep[0] = 4 * pp + 2;
              t.need[0] = bs[pp].nC;
            }
          } else if (pass == 1) {
            t.dep[0] = 4 * (int)bi;
            t.need[0] = b.nA;
          } else if (pass == 2) {
            t.dep[0] = 4 * (int)bi + 1;
            t.need[0] = b.nB;
            const int po = prev_overlap(bi);
            if (po >= 0) {
              t.dep[1] = 4 * po + 2;
              t.need[1] = bs[po].nC;
            }
            const int pp = prev_same_plan(bi);
            if (pp >= 0 && bs[pp].fin) {
              t.dep[2] = 4 * pp + 3;
              t.need[2] = 1;
            }
          } else {
            t.dep[0] = 4 * (int)bi + 2;
            t.need[0] = b.nC;
            if (fin_prev >= 0) {
              t.dep[1] = fin_prev;
              t.need[1] = 1;
            }
            fin_prev = 4 * (int)bi + 3;
          }
          out.push_back(t);
        }
      }
    }
  }
  return out;
}

}  // namespace kx
