// Host instantiation of the device term sweep (ph_sweep.hpp) with a symbolic
// number type that records every multiplication, to check the product
// sequence against Table 6 of the paper.  Usage: sweep_symbolic k e1 ... ek
#include <cstdio>
#include <cstdlib>
#include <string>
#include <vector>

#include "ph_sweep.hpp"

struct Sym {
    std::vector<int> e;  // exponent of each variable
    bool coef = false;   // the term's coefficient (or a power of it)
};

static std::vector<std::string> g_log;

static std::string name(const Sym &s)
{
    std::string r;
    for (size_t v = 0; v < s.e.size(); ++v)
        for (int k = 0; k < s.e[v]; ++k) r += (r.empty() ? "" : "*") + std::string("a") + std::to_string(v + 1);
    return r.empty() ? "1" : r;
}

Sym num_mul(const Sym &a, const Sym &b)
{
    Sym r;
    r.e.resize(8, 0);
    for (int v = 0; v < 8; ++v) r.e[v] = a.e[v] + b.e[v];
    r.coef = false;
    // a product with the coefficient itself folds c into the partial
    // products; the others belong to the bare variable product of Table 6
    g_log.push_back((a.coef || b.coef ? "c " : "") + name(r));
    return r;
}

Sym num_scale(const Sym &a, double) { return a; }

int main(int argc, char **argv)
{
    const int k = argc > 1 ? std::atoi(argv[1]) : 4;
    uint32_t fw[8];
    for (int l = 0; l < k; ++l) {
        const int e = argc > 2 + l ? std::atoi(argv[2 + l]) : 1;
        fw[l] = uint32_t(l) | (uint32_t(e) << 16);
    }
    Sym c;
    c.e.assign(8, 0);
    c.coef = true;
    auto X = [](int var) {
        Sym s;
        s.e.assign(8, 0);
        s.e[var] = 1;
        return s;
    };
    std::vector<std::string> parts(k);
    Sym v = ph::term_sweep<8, true>(k, fw, c, X, [&](int l, uint32_t, const Sym &p) { parts[l] = name(p); });
    for (auto &s : g_log) std::printf("%s\n", s.c_str());
    for (int l = 0; l < k; ++l) std::printf("d%d %s\n", l + 1, parts[l].c_str());
    std::printf("value %s\n", name(v).c_str());
    return 0;
}
