// Host driver for the sanitizer build of the load-balancing planner (test
// infrastructure).  Built with g++ -fsanitize=address,undefined together with
// the planner's source by tests/test_host_sanitizers.py.  Reads cases from a
// text file:
//   n_cases
//   n_proc min_frac max_ops   (then, per process) n_prob cost_0 .. cost_{n_prob-1}
// and prints per case "case <i> rc <rc> n_ops <k>", one line per emitted
// operation "op sender receiver first count load planned" and one line
// "loads l_0 .. l_{n_proc-1}" (%.17g), for comparison with the regular build.
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "../../include/chem.h"

int main(int argc, char **argv) {
    if (argc != 2) {
        fprintf(stderr, "usage: %s cases.txt\n", argv[0]);
        return 2;
    }
    FILE *f = fopen(argv[1], "r");
    if (!f) return 2;
    int n_cases = 0;
    if (fscanf(f, "%d", &n_cases) != 1) return 2;
    for (int c = 0; c < n_cases; ++c) {
        int n_proc = 0;
        double min_frac = 0.0;
        long long max_ops = 0;
        if (fscanf(f, "%d %lf %lld", &n_proc, &min_frac, &max_ops) != 3) return 2;
        std::vector<int64_t> n_prob((size_t)(n_proc > 0 ? n_proc : 0));
        std::vector<double> cost;
        cost.reserve(1);   // a valid (non-null) cost array also when there are no problems
        for (int i = 0; i < n_proc; ++i) {
            long long k = 0;
            if (fscanf(f, "%lld", &k) != 1) return 2;
            n_prob[(size_t)i] = k;
            for (long long j = 0; j < k; ++j) {
                double t = 0.0;
                if (fscanf(f, "%lf", &t) != 1) return 2;
                cost.push_back(t);
            }
        }
        // exact-size buffers, so that a write past max_ops or n_proc is caught
        std::vector<chem_balance_op> ops((size_t)(max_ops > 0 ? max_ops : 0));
        std::vector<double> loads((size_t)(n_proc > 0 ? n_proc : 0));
        int64_t n_ops = -1;
        const int rc = chem_plan_balance(n_proc, n_prob.data(), cost.data(), min_frac,
                                         ops.empty() ? nullptr : ops.data(), max_ops, &n_ops,
                                         loads.empty() ? nullptr : loads.data());
        printf("case %d rc %d n_ops %lld\n", c, rc, (long long)n_ops);
        if (rc != 0) continue;
        for (long long i = 0; i < n_ops && i < max_ops; ++i) {
            const chem_balance_op &o = ops[(size_t)i];
            printf("op %d %d %lld %lld %.17g %.17g\n", o.sender, o.receiver, (long long)o.first,
                   (long long)o.count, o.load, o.planned);
        }
        printf("loads");
        for (double l : loads) printf(" %.17g", l);
        printf("\n");
    }
    fclose(f);
    return 0;
}
