// HEGMM-En planner; see planner.h.
#include "planner.h"

#include <algorithm>
#include <map>
#include <set>
#include <stdexcept>

namespace hg {

namespace {

struct Consts { int d, M, K, W; };

Consts constants(int mo, int lb, int no) {
    Consts c;
    c.d = mo < lb ? (lb + mo - 1) / mo : 1;  // Theorem 5: ceil(l/m) copies when m < l
    c.M = c.d * mo;
    c.K = std::min(mo, lb);                  // p = min(m, l, n) loop trips (Algorithm 2)
    c.W = std::max(lb, no);                  // packed width max(l, N) of the left operand
    return c;
}

// Add the diagonals found in `cand` (z -> slot list) in the order given; a
// lone diagonal that covers the whole M x no region needs no mask.
void add_terms(Plan &p, std::vector<Term> &out, std::map<int, std::vector<int>> &cand,
               const int order[2], int S, size_t region) {
    std::vector<std::pair<int, std::vector<int> *>> found;
    for (int i = 0; i < 2; ++i) {
        auto it = cand.find(order[i]);
        if (it != cand.end() && !it->second.empty()) found.push_back({order[i], &it->second});
    }
    if (found.size() == 1 && found[0].second->size() == region) {
        out.push_back({found[0].first, -1});
        return;
    }
    for (auto &f : found) {
        std::vector<uint8_t> bm(S, 0);
        for (int s : *f.second) bm[s] = 1;
        p.masks.push_back(std::move(bm));
        out.push_back({f.first, (int)p.masks.size() - 1});
    }
}

// Every diagonal found, in increasing z; a lone diagonal covering the whole
// region needs no mask.
void add_all_terms(Plan &p, std::vector<Term> &out, const std::map<int, std::vector<int>> &cand, int S,
                   size_t region) {
    if (cand.size() == 1 && cand.begin()->second.size() == region) {
        out.push_back({cand.begin()->first, -1});
        return;
    }
    for (auto &kv : cand) {
        std::vector<uint8_t> bm(S, 0);
        for (int s : kv.second) bm[s] = 1;
        p.masks.push_back(std::move(bm));
        out.push_back({kv.first, (int)p.masks.size() - 1});
    }
}

// Algorithm 1's transforms on column-major sigma(X) (mo x l) and tau(Y)
// (l x no): output (i, j) reads slot i + ((j + k) mod l) mo, resp.
// ((i + k) mod l) + j l; the diagonal is the difference of the slots.
std::map<int, std::vector<int>> alg1_eps(int mo, int l, int no, int k) {
    std::map<int, std::vector<int>> cand;
    for (int j = 0; j < no; ++j)
        for (int i = 0; i < mo; ++i) {
            const int dst = i + j * mo;
            cand[i + ((j + k) % l) * mo - dst].push_back(dst);
        }
    return cand;
}

std::map<int, std::vector<int>> alg1_omega(int mo, int l, int no, int k) {
    std::map<int, std::vector<int>> cand;
    for (int j = 0; j < no; ++j)
        for (int i = 0; i < mo; ++i) {
            const int dst = i + j * mo;
            cand[((i + k) % l) + j * l - dst].push_back(dst);
        }
    return cand;
}

// sigma on X (mo x l) and tau on Y (l x no), both column-major: output
// slot i + j mo reads i + ((i + j) mod l) mo, resp. slot i + j l reads
// ((i + j) mod l) + j l (the Section III-A definitions).
std::map<int, std::vector<int>> sigma_diags(int mo, int l) {
    std::map<int, std::vector<int>> cand;
    for (int j = 0; j < l; ++j)
        for (int i = 0; i < mo; ++i) {
            const int dst = i + j * mo;
            cand[i + ((i + j) % l) * mo - dst].push_back(dst);
        }
    return cand;
}

std::map<int, std::vector<int>> tau_diags(int l, int no) {
    std::map<int, std::vector<int>> cand;
    for (int j = 0; j < no; ++j)
        for (int i = 0; i < l; ++i) {
            const int dst = i + j * l;
            cand[((i + j) % l) + j * l - dst].push_back(dst);
        }
    return cand;
}

long long alg1_switched(int mo, int l, int no, int S) {
    long long c = 0;
    for (int k = 0; k < l; ++k) {
        for (auto &kv : alg1_eps(mo, l, no, k)) c += (((kv.first % S) + S) % S) != 0;
        for (auto &kv : alg1_omega(mo, l, no, k)) c += (((kv.first % S) + S) % S) != 0;
    }
    return c;
}

Plan make_plan_alg1(int m, int l, int n, int S, bool cloud) {
    if ((long long)m * l > S || (long long)l * n > S || (long long)m * n > S)
        throw std::range_error("shape does not fit one ciphertext row");
    Plan p;
    p.method = 1;
    p.m = m; p.l = l; p.n = n;
    p.transposed = alg1_switched(n, l, m, S) < alg1_switched(m, l, n, S);
    p.mo = p.transposed ? n : m;
    p.no = p.transposed ? m : n;
    p.nb = 1; p.lb = l; p.d = 1; p.M = p.mo; p.K = l; p.W = l;
    const size_t region = (size_t)p.mo * p.no;
    for (int k = 0; k < l; ++k) {
        std::vector<Term> e, w;
        add_all_terms(p, e, alg1_eps(p.mo, l, p.no, k), S, region);
        add_all_terms(p, w, alg1_omega(p.mo, l, p.no, k), S, region);
        p.eps.push_back(e);
        p.omega.push_back(w);
    }
    p.fold.push_back(0);
    if (cloud) {
        p.method = 3;
        add_all_terms(p, p.sigma, sigma_diags(p.mo, l), S, (size_t)p.mo * l);
        add_all_terms(p, p.tau, tau_diags(l, p.no), S, (size_t)l * p.no);
    }
    return p;
}

}  // namespace

Plan make_plan(int m, int l, int n, int S, int method, int min_blocks) {
    if (m <= 0 || l <= 0 || n <= 0) throw std::invalid_argument("dimensions must be positive");
    if (min_blocks > 1 && method != 2) throw std::invalid_argument("forced blocking needs HEGMM-En");
    if (method == 1 || method == 3) return make_plan_alg1(m, l, n, S, method == 3);
    if (method != 2) throw std::invalid_argument("method must be 1, 2 or 3");
    Plan p;
    p.m = m; p.l = l; p.n = n;
    // Orientation in Algorithm 2's order: p == m duplicates A; else p == n
    // duplicates B, realised as the transposed problem B^T A^T; else no
    // duplication.
    int pm = std::min(m, std::min(l, n));
    p.transposed = (pm != m) && (pm == n);
    p.mo = p.transposed ? n : m;
    p.no = p.transposed ? m : n;

    auto fits = [&](int lb) {
        Consts c = constants(p.mo, lb, p.no);
        return (long long)c.M * c.W <= S;
    };
    // the fewest inner blocks (at least min_blocks, at most l) whose block
    // length fits
    int nb = std::min(std::max(min_blocks, 1), l);
    while (nb <= l && !fits((l + nb - 1) / nb)) ++nb;
    if (nb > l) throw std::range_error("shape does not fit one ciphertext row");
    p.nb = nb;
    p.lb = (l + nb - 1) / nb;
    Consts c = constants(p.mo, p.lb, p.no);
    p.d = c.d; p.M = c.M; p.K = c.K; p.W = c.W;
    const int M = p.M, mo = p.mo, no = p.no, lb = p.lb, W = p.W;
    const size_t region = (size_t)M * no;

    for (int k = 0; k < p.K; ++k) {
        // eps^k: output (i, j) takes source column c = j + k (j + k - lb once
        // past the packed width), a left rotation by (c - j) * M.  Row block
        // h = i / mo carries partial product (k + h*mo) mod lb (Theorem 5) and
        // is masked out when h*mo + k >= lb, so no partial product is added
        // twice.
        std::map<int, std::vector<int>> cand;
        for (int j = 0; j < no; ++j) {
            int cc = j + k < W ? j + k : j + k - lb;
            int z = (cc - j) * M;
            for (int i = 0; i < M; ++i) {
                if ((i / mo) * mo + k >= lb) continue;
                cand[z].push_back(i + j * M);
            }
        }
        std::vector<Term> e;
        int eo[2] = {k * M, (k - lb) * M};
        add_terms(p, e, cand, eo, S, region);
        p.eps.push_back(e);
        // omega^k: output (i, j) takes source row r = i + k (i + k - lb past M).
        cand.clear();
        for (int j = 0; j < no; ++j)
            for (int i = 0; i < M; ++i) {
                int r = i + k < M ? i + k : i + k - lb;
                cand[r - i].push_back(i + j * M);
            }
        std::vector<Term> w;
        int wo[2] = {k, k - lb};
        add_terms(p, w, cand, wo, S, region);
        p.omega.push_back(w);
    }
    for (int h = 0; h < p.d; ++h) p.fold.push_back(h * mo);
    return p;
}

std::vector<int> Plan::rotations(int S) const {
    std::set<int> zs;
    auto addz = [&](int z) {
        int r = ((z % S) + S) % S;
        if (r) zs.insert(r);
    };
    for (auto &v : eps) for (auto &t : v) addz(t.z);
    for (auto &v : omega) for (auto &t : v) addz(t.z);
    for (auto &t : sigma) addz(t.z);
    for (auto &t : tau) addz(t.z);
    for (int z : fold) addz(z);
    return std::vector<int>(zs.begin(), zs.end());
}

int Plan::key_switched_terms(int S) const {
    int c = 0;
    auto cnt = [&](const std::vector<Term> &v) {
        for (auto &t : v) c += (((t.z % S) + S) % S) != 0;
    };
    for (int b = 0; b < nb; ++b) {
        for (auto &v : eps) cnt(v);
        for (auto &v : omega) cnt(v);
    }
    cnt(sigma);
    cnt(tau);
    for (int z : fold) c += (((z % S) + S) % S) != 0;
    return c;
}

std::vector<uint64_t> pack_operand(const Plan &p, int side, const int64_t *X, int block, uint64_t t, int S) {
    std::vector<uint64_t> v(S, 0);
    auto modt = [&](int64_t x) -> uint64_t {
        int64_t r = x % (int64_t)t;
        return (uint64_t)(r < 0 ? r + (int64_t)t : r);
    };
    const int lo = block * p.lb;
    if (p.method == 3) {
        // Xo (mo x l) and Yo (l x no) as they are, column-major: sigma and
        // tau are applied to the ciphertexts
        if (side == 0) {
            for (int i = 0; i < p.mo; ++i)
                for (int c = 0; c < p.l; ++c)
                    v[i + (size_t)c * p.mo] = modt(p.transposed ? X[(size_t)c * p.n + i] : X[(size_t)i * p.l + c]);
        } else {
            for (int r = 0; r < p.l; ++r)
                for (int j = 0; j < p.no; ++j)
                    v[r + (size_t)j * p.l] = modt(p.transposed ? X[(size_t)j * p.l + r] : X[(size_t)r * p.n + j]);
        }
        return v;
    }
    if (p.method == 1) {
        // Algorithm 1: sigma(Xo) (mo x l) and tau(Yo) (l x no), column-major
        if (side == 0) {
            for (int i = 0; i < p.mo; ++i)
                for (int c = 0; c < p.l; ++c) {
                    const int cc = (i + c) % p.l;
                    v[i + (size_t)c * p.mo] = modt(p.transposed ? X[(size_t)cc * p.n + i] : X[(size_t)i * p.l + cc]);
                }
        } else {
            for (int r = 0; r < p.l; ++r)
                for (int j = 0; j < p.no; ++j) {
                    const int rr = (r + j) % p.l;
                    v[r + (size_t)j * p.l] = modt(p.transposed ? X[(size_t)j * p.l + rr] : X[(size_t)rr * p.n + j]);
                }
        }
        return v;
    }
    // entries of the oriented operands, zero outside the block
    if (side == 0) {
        // left operand Xo (mo x l): A itself, or B^T when transposed (X = B, l x n)
        auto xo = [&](int i, int c) -> int64_t {
            int cg = lo + c;
            if (cg >= p.l) return 0;
            return p.transposed ? X[(size_t)cg * p.n + i] : X[(size_t)i * p.l + cg];
        };
        // x[i + c*M] = Xb[i mod mo][(i + c) mod lb]: eps^0_{M x W}(sigma(Xbar))
        for (int i = 0; i < p.M; ++i)
            for (int c = 0; c < p.W; ++c)
                v[i + (size_t)c * p.M] = modt(xo(i % p.mo, (i + c) % p.lb));
    } else {
        // right operand Yo (l x no): B itself, or A^T when transposed (X = A, m x l)
        auto yo = [&](int r, int j) -> int64_t {
            int rg = lo + r;
            if (rg >= p.l) return 0;
            return p.transposed ? X[(size_t)j * p.l + rg] : X[(size_t)rg * p.n + j];
        };
        // y[r + j*M] = Yb[(r + j) mod lb][j]: omega^0_{M x no}(tau(Yb))
        for (int r = 0; r < p.M; ++r)
            for (int j = 0; j < p.no; ++j)
                v[r + (size_t)j * p.M] = modt(yo((r + j) % p.lb, j));
    }
    return v;
}

}  // namespace hg
