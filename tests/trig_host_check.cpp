// Host build of the kernels' sin/cos routine (cf_sincos): reads float64
// arguments (one per line, as C99 hex floats) and prints sin x and cos x in
// the same form.
#include <cstdio>
#include <cstdlib>

#include "trig.hpp"

int main() {
    char buf[128];
    while (std::fgets(buf, sizeof buf, stdin)) {
        const double x = std::strtod(buf, nullptr);
        double s, c;
        chessfad::cf_sincos(x, &s, &c);
        std::printf("%a %a\n", s, c);
    }
    return 0;
}
