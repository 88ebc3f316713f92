// Pieces shared by the kernel generators: the text buffer, exact spelling of
// doubles, Taylor coefficients of 2^f and the species of each reaction.
// Host-side only.
#pragma once
#include <algorithm>
#include <cstdarg>
#include <cstdio>
#include <string>
#include <vector>

#include "ak_jit.h"

namespace ak {

struct Text {
    std::string s;
    void operator()(const char *fmt, ...) __attribute__((format(printf, 2, 3)))
    {
        char buf[1024];
        va_list ap;
        va_start(ap, fmt);
        const int n = vsnprintf(buf, sizeof buf, fmt, ap);
        va_end(ap);
        if (n >= (int)sizeof buf) {
            std::vector<char> big(n + 1);
            va_start(ap, fmt);
            vsnprintf(big.data(), big.size(), fmt, ap);
            va_end(ap);
            s.append(big.data(), n);
        } else {
            s.append(buf, n);
        }
    }
};

// exact decimal-free spelling of a double for the generated text
inline std::string lit(double x)
{
    char b[64];
    snprintf(b, sizeof b, "%a", x);
    return b;
}

// ln(2)^k / k!, the Taylor coefficients of 2^f, rounded to double
inline std::vector<double> exp2_taylor(int deg)
{
    std::vector<double> c(deg + 1);
    long double t = 1.0L;
    const long double ln2 = 0.693147180559945309417232121458176568L;
    for (int k = 0; k <= deg; ++k) {
        c[k] = (double)t;
        t = t * ln2 / (long double)(k + 1);
    }
    return c;
}

// Species of each reaction, each once.
inline std::vector<std::vector<int>> reaction_species(const JitMech &m)
{
    std::vector<std::vector<int>> rs(m.nr);
    for (int j = 0; j < m.nr; ++j)
        for (int i = 0; i < m.aux[j].nf + m.aux[j].nr; ++i) {
            const int k = m.aux[j].sp[i];
            if (std::find(rs[j].begin(), rs[j].end(), k) == rs[j].end()) rs[j].push_back(k);
        }
    return rs;
}

}  // namespace ak
