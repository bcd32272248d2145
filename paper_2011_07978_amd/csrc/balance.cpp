// Load-balancing plan across processes: Algorithm 1 of Sec. 2.2 (host only).
//
// Loads are the summed costs of each process's problems; processes are
// sorted by load and a receiver pointer (lightest) and a sender pointer
// (heaviest) walk towards each other, pairing them to move min(mean -
// receiver load, sender load - mean) of load at a time.  The load moved is
// turned into a count of the sender's problems (in its list order, from where
// its previous emitted send stopped, the shortest prefix whose cost reaches
// the planned load).  Pairs that would move less than min_frac of the mean
// load are planned but not emitted.
#include <math.h>
#include <stdint.h>

#include <algorithm>
#include <numeric>
#include <vector>

#include "../../include/chem.h"

extern "C" int chem_plan_balance(int32_t n_proc, const int64_t *n_prob, const double *t_cost,
                                 double min_frac, chem_balance_op *ops, int64_t max_ops,
                                 int64_t *n_ops, double *loads_after) {
    if (n_proc < 1 || !n_prob || !n_ops || (max_ops > 0 && !ops) || max_ops < 0 ||
        !(min_frac >= 0.0))
        return CHEM_E_INVALID_ARG;
    std::vector<int64_t> off((size_t)n_proc + 1, 0);
    for (int k = 0; k < n_proc; ++k) {
        if (n_prob[k] < 0) return CHEM_E_INVALID_ARG;
        off[k + 1] = off[k] + n_prob[k];
    }
    if (off[n_proc] > 0 && !t_cost) return CHEM_E_INVALID_ARG;
    std::vector<double> l((size_t)n_proc, 0.0);
    for (int k = 0; k < n_proc; ++k)
        for (int64_t q = off[k]; q < off[k + 1]; ++q) {
            const double t = t_cost[q];
            if (!(t >= 0.0) || !isfinite(t)) return CHEM_E_INVALID_ARG;
            l[k] += t;
        }
    double mean = 0.0;
    for (int k = 0; k < n_proc; ++k) mean += l[k];
    mean /= n_proc;

    std::vector<int> R((size_t)n_proc);
    std::iota(R.begin(), R.end(), 0);
    std::stable_sort(R.begin(), R.end(), [&](int a, int b) { return l[a] < l[b]; });
    std::vector<double> L((size_t)n_proc);
    for (int i = 0; i < n_proc; ++i) L[i] = l[R[i]];

    std::vector<double> after(l);
    std::vector<int64_t> cursor((size_t)n_proc, 0);   // next problem of each sender
    int64_t emitted = 0;
    int i = 0, j = n_proc - 1;
    while (i != j) {
        const double dL = std::min(mean - L[i], L[j] - mean);
        const int rr = R[i], rs = R[j];
        // shortest prefix of the sender's remaining problems reaching dL
        const int64_t first = cursor[rs];
        int64_t cnt = 0;
        double sent = 0.0;
        while (first + cnt < n_prob[rs] && sent < dL) sent += t_cost[off[rs] + first + cnt++];
        if (dL >= min_frac * mean && cnt > 0) {
            if (emitted < max_ops) ops[emitted] = chem_balance_op{rs, rr, first, cnt, sent, dL};
            ++emitted;
            cursor[rs] += cnt;
            after[rs] -= sent;
            after[rr] += sent;
        }
        L[i] += dL;
        L[j] -= dL;
        if (fabs(L[i] - mean) <= 1e-12 * mean) ++i;
        else --j;
    }
    *n_ops = emitted;
    if (loads_after)
        for (int k = 0; k < n_proc; ++k) loads_after[k] = after[k];
    return emitted > max_ops ? CHEM_E_INVALID_ARG : CHEM_OK;
}
