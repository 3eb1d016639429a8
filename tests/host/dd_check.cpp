// Evaluates the double-double functions of fsa_dd.hpp on the host for the
// test suite: reads "op x_hi x_lo [y_hi y_lo]" lines, prints "hi lo" with
// full precision.
#include <cstdio>
#include <cstring>

#include "../../paper_2504_19410_amd/csrc/fsa_dd.hpp"

using fsa::dd;

int main() {
    char op[32];
    double a, b, c, e;
    while (std::scanf("%31s %la %la %la %la", op, &a, &b, &c, &e) == 5) {
        const dd x = fsa::dd_make(a, b), y = fsa::dd_make(c, e);
        dd r = fsa::dd_of(0.0), r2 = fsa::dd_of(0.0);
        if (!std::strcmp(op, "add")) r = x + y;
        else if (!std::strcmp(op, "mul")) r = x * y;
        else if (!std::strcmp(op, "div")) r = x / y;
        else if (!std::strcmp(op, "divd")) r = x / c;
        else if (!std::strcmp(op, "sqrt")) r = fsa::dd_sqrt(x);
        else if (!std::strcmp(op, "exp")) r = fsa::dd_exp(x);
        else if (!std::strcmp(op, "expm1")) r = fsa::dd_expm1(x);
        else if (!std::strcmp(op, "erf")) r = fsa::dd_erf(x);
        else if (!std::strcmp(op, "sincos")) fsa::dd_sincos_turn(a, &r, &r2);
        std::printf("%a %a %a %a\n", r.hi, r.lo, r2.hi, r2.lo);
    }
    return 0;
}
