// Host driver for the sanitizer build of the library's mechanism check (test
// infrastructure).  tests/test_host_sanitizers.py compiles the host side of
// csrc/api.cpp with AddressSanitizer and UBSan, links it with this driver and
// the library's other (unsanitized) objects, and runs chem_validate_mechanism
// -- the host-only check chem_set_mechanism runs before any upload -- on each
// mechanism file named on the command line, printing "rc <code> <message>".
//
// File layout (little-endian, written by the test):
//   int32 E, N, R, n_eff, has_falloff, has_plog
//   f64 elem_mass[E]; i32 comp[N*E]; f64 W[N]; f64 nasa[N*7];
//   i32 reac[R*2]; i32 prod[R*3]; f64 A[R], b[R], Ea[R]; i32 tb[R];
//   i32 eff_r[n_eff], eff_s[n_eff]; f64 eff_v[n_eff];
//   (has_falloff) i32 falloff[R]; f64 falloff_params[R*7];
//   (has_plog) i32 plog_count[R]; f64 plog_params[R*32]
#include <stdint.h>
#include <stdio.h>

#include <vector>

#include "../../include/chem.h"

// (arrays are never null, also when empty, as from the library's binding)
template <typename T>
static bool rd(FILE *f, std::vector<T> &v, size_t n) {
    v.reserve(n ? n : 1);
    v.resize(n);
    return n == 0 || fread(v.data(), sizeof(T), n, f) == n;
}

int main(int argc, char **argv) {
    for (int a = 1; a < argc; ++a) {
        FILE *f = fopen(argv[a], "rb");
        if (!f) return 2;
        std::vector<int32_t> hdr, comp, reac, prod, tb, eff_r, eff_s, fo, plog_n;
        std::vector<double> elem, W, nasa, A, b, Ea, eff_v, fop, plog;
        if (!rd(f, hdr, 6)) return 2;
        const size_t E = (size_t)hdr[0], N = (size_t)hdr[1], R = (size_t)hdr[2];
        const size_t ne = (size_t)hdr[3];
        bool ok = rd(f, elem, E) && rd(f, comp, N * E) && rd(f, W, N) && rd(f, nasa, N * 7) &&
                  rd(f, reac, R * 2) && rd(f, prod, R * 3) && rd(f, A, R) && rd(f, b, R) &&
                  rd(f, Ea, R) && rd(f, tb, R) && rd(f, eff_r, ne) && rd(f, eff_s, ne) &&
                  rd(f, eff_v, ne);
        if (ok && hdr[4]) ok = rd(f, fo, R) && rd(f, fop, R * 7);
        if (ok && hdr[5]) ok = rd(f, plog_n, R) && rd(f, plog, R * 32);
        fclose(f);
        if (!ok) return 2;
        chem_mech_desc d{};
        d.n_elements = hdr[0];
        d.n_species = hdr[1];
        d.n_reactions = hdr[2];
        d.elem_mass = elem.data();
        d.composition = comp.data();
        d.W = W.data();
        d.nasa = nasa.data();
        d.reactants = reac.data();
        d.products = prod.data();
        d.A = A.data();
        d.b = b.data();
        d.Ea = Ea.data();
        d.third_body = tb.data();
        d.n_eff = hdr[3];
        d.eff_reaction = eff_r.data();
        d.eff_species = eff_s.data();
        d.eff_value = eff_v.data();
        d.falloff = hdr[4] ? fo.data() : nullptr;
        d.falloff_params = hdr[4] ? fop.data() : nullptr;
        d.plog_count = hdr[5] ? plog_n.data() : nullptr;
        d.plog_params = hdr[5] ? plog.data() : nullptr;
        char msg[512];
        msg[0] = '\0';
        const int rc = chem_validate_mechanism(&d, msg, (int32_t)sizeof msg);
        printf("rc %d %s\n", rc, msg);
    }
    return 0;
}
