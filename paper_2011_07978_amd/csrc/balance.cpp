// Load-balancing plan across processes (Algorithm 1, Sec. 2.2), host only.
//
// The goal of the paper's plan: every process should end at the mean load,
// heavy processes giving problems to light ones, and moves worth less than a
// small fraction of the mean are not made.  Its pairing of the lightest
// remaining receiver with the heaviest remaining sender is the north-west
// corner rule of a transportation problem, which is how it is built here:
//   - receivers (load below the mean) are laid out lightest first as
//     consecutive intervals of length mean - load on one axis, senders (load
//     above the mean) heaviest first as intervals of length load - mean on
//     another; both axes end at the total imbalance;
//   - every overlap of a receiver interval with a sender interval is one
//     planned transfer of that length, found by merging the two sorted
//     sequences of interval ends (a receiver and a sender ending together, to
//     1e-12 of the mean, retire the receiver first);
//   - a transfer below min_frac of the mean, or not above 1e-12 of it, is
//     dropped; each kept transfer becomes a count of the sender's problems,
//     taken in its list order from where its previous transfer stopped: the
//     fewest whose cost reaches the planned load (all that remain if none do).
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/chem.h"

namespace {

// One side of the transportation problem: processes and the cumulative ends
// of their intervals.
struct Side {
    std::vector<int> proc;
    std::vector<double> end;
};

}  // namespace

extern "C" int chem_plan_balance(int32_t n_proc, const int64_t *n_prob, const double *t_cost,
                                 double min_frac, chem_balance_op *ops, int64_t max_ops,
                                 int64_t *n_ops, double *loads_after) {
    if (n_proc < 1 || !n_prob || !n_ops || (max_ops > 0 && !ops) || max_ops < 0 ||
        !(min_frac >= 0.0))
        return CHEM_E_INVALID_ARG;
    std::vector<int64_t> start((size_t)n_proc + 1, 0);
    for (int k = 0; k < n_proc; ++k) {
        if (n_prob[k] < 0) return CHEM_E_INVALID_ARG;
        start[k + 1] = start[k] + n_prob[k];
    }
    if (start[n_proc] > 0 && !t_cost) return CHEM_E_INVALID_ARG;
    for (int64_t q = 0; q < start[n_proc]; ++q)
        if (!(t_cost[q] >= 0.0) || !isfinite(t_cost[q])) return CHEM_E_INVALID_ARG;

    std::vector<double> load((size_t)n_proc, 0.0);
    double total = 0.0;
    for (int k = 0; k < n_proc; ++k) {
        for (int64_t q = start[k]; q < start[k + 1]; ++q) load[k] += t_cost[q];
        total += load[k];
    }
    const double mean = total / n_proc;
    const double tie = 1e-12 * mean;

    // processes by ascending load (ties by index): receivers from the light
    // end, senders from the heavy end
    std::vector<int> by_load((size_t)n_proc);
    std::iota(by_load.begin(), by_load.end(), 0);
    std::stable_sort(by_load.begin(), by_load.end(), [&](int a, int b) { return load[a] < load[b]; });
    Side rec, snd;
    double acc = 0.0;
    for (int k : by_load)
        if (load[k] < mean) {
            acc += mean - load[k];
            rec.proc.push_back(k);
            rec.end.push_back(acc);
        }
    acc = 0.0;
    for (auto it = by_load.rbegin(); it != by_load.rend(); ++it)
        if (load[*it] > mean) {
            acc += load[*it] - mean;
            snd.proc.push_back(*it);
            snd.end.push_back(acc);
        }

    std::vector<double> after(load);
    std::vector<int64_t> next((size_t)n_proc, 0);   // each sender's first problem not yet given
    int64_t emitted = 0;
    double x = 0.0;                                  // position on the merged axis
    size_t a = 0, b = 0;
    while (a < rec.proc.size() && b < snd.proc.size()) {
        const double stop = std::min(rec.end[a], snd.end[b]);
        const double planned = stop - x;
        const int r = rec.proc[a], s = snd.proc[b];
        if (planned >= min_frac * mean && planned > tie) {
            const int64_t *n_s = n_prob + s;
            const double *t = t_cost + start[s];
            const int64_t first = next[s];
            int64_t q = first;
            double moved = 0.0;
            while (q < *n_s && moved < planned) moved += t[q++];
            if (q > first) {
                if (emitted < max_ops) ops[emitted] = chem_balance_op{s, r, first, q - first, moved, planned};
                ++emitted;
                next[s] = q;
                after[s] -= moved;
                after[r] += moved;
            }
        }
        x = stop;
        // retire the interval that ends here; the receiver first on a tie
        if (rec.end[a] <= snd.end[b] + tie) ++a;
        else ++b;
    }
    *n_ops = emitted;
    if (loads_after)
        for (int k = 0; k < n_proc; ++k) loads_after[k] = after[k];
    return emitted > max_ops ? CHEM_E_INVALID_ARG : CHEM_OK;
}
