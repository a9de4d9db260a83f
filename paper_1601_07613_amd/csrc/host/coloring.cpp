// Face coloring of Section 3.1 (modified greedy + conflict resolution) and
// the standard greedy coloring of Section 1.
//
// The paper leaves its random choices and the loop rule open.  This file
// follows one written specification, stated in the header of the public
// API: SplitMix64 draws, choose(list) = list[0] for one element, else
// list[next() % len]; candidates listed left element first in local face
// order; a loop is a conflict whose swap candidates have all been visited by
// the current chain.  Colors are kept as bit masks per element.
#include <chrono>
#include <deque>

#include "internal.hpp"

namespace dgc {

namespace {

struct SplitMix64 {
    uint64_t s;
    explicit SplitMix64(uint64_t seed) : s(seed) {}
    uint64_t next() {
        s += 0x9E3779B97F4A7C15ull;
        uint64_t z = s;
        z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
        z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
        return z ^ (z >> 31);
    }
    template <class T>
    T choose(const T *items, int n) {
        if (n == 1) return items[0];
        return items[next() % (uint64_t)n];
    }
};

struct Colorer {
    Mesh &m;
    std::vector<int8_t> &color;
    int F;

    Colorer(Mesh &mesh, std::vector<int8_t> &c) : m(mesh), color(c), F(mesh.F) {}

    unsigned used(int64_t e) const {
        if (e < 0) return 0u;
        unsigned u = 0;
        const int32_t *fa = &m.elem_face[e * m.max_slots];
        for (int k = 0; k < F; ++k) {
            if (fa[k] < 0) continue;  // padded slot (an element with fewer faces)
            int8_t c = color[fa[k]];
            if (c >= 0) u |= 1u << c;
        }
        return u;
    }
    // ascending list of the colors in mask; returns the count
    int list_of(unsigned mask, int8_t *out) const {
        int n = 0;
        for (int c = 0; c < F; ++c)
            if (mask & (1u << c)) out[n++] = (int8_t)c;
        return n;
    }
};

}  // namespace

dgc_status color_paper(Mesh &m, uint64_t seed, int64_t max_swaps, dgc_color_stats *st) {
    const int F = m.F;
    const int64_t E = m.E;
    const unsigned full = (1u << F) - 1u;
    std::vector<int8_t> color(E, -1);
    Colorer C(m, color);
    SplitMix64 rng(seed);
    if (max_swaps < 0) max_swaps = 1000 * E;
    int8_t buf[DGC_MAX_COLORS];

    // stage 1: modified greedy
    for (int64_t f = 0; f < E; ++f) {
        unsigned av = full & ~(C.used(m.face_L[f]) | C.used(m.face_R[f]));
        int n = C.list_of(av, buf);
        if (n > 0) color[f] = rng.choose(buf, n);
    }
    std::deque<int64_t> queue;
    for (int64_t f = 0; f < E; ++f)
        if (color[f] < 0) queue.push_back(f);
    dgc_color_stats s{};
    s.conflicts_after_greedy = (int64_t)queue.size();

    // stage 2: conflict resolution
    std::vector<int64_t> stamp(E, -1);  // chain id that visited each face
    int64_t chain = 0, moves = 0;
    int64_t cand[2 * 8], unv[2 * 8];
    while (!queue.empty()) {
        int64_t f = queue.front();
        queue.pop_front();
        if (color[f] >= 0) continue;
        ++chain;
        stamp[f] = chain;
        int64_t cur = f;
        for (;;) {
            const int64_t lc = m.face_L[cur], rc = m.face_R[cur];
            const unsigned uL = C.used(lc), uR = C.used(rc);
            unsigned av = full & ~(uL | uR);
            if (av) {
                int n = C.list_of(av, buf);
                color[cur] = rng.choose(buf, n);
                break;
            }
            int nc = 0;
            const int32_t *fl = &m.elem_face[lc * m.max_slots];
            for (int k = 0; k < F; ++k) {
                int64_t g = fl[k];
                if (g >= 0 && g != cur && color[g] >= 0 && !(uR & (1u << color[g]))) cand[nc++] = g;
            }
            if (rc >= 0) {
                const int32_t *fr = &m.elem_face[rc * m.max_slots];
                for (int k = 0; k < F; ++k) {
                    int64_t g = fr[k];
                    if (g >= 0 && g != cur && color[g] >= 0 && !(uL & (1u << color[g]))) cand[nc++] = g;
                }
            }
            int nu = 0;
            for (int k = 0; k < nc; ++k)
                if (stamp[cand[k]] != chain) unv[nu++] = cand[k];
            if (moves >= max_swaps) {
                if (st) *st = s;
                return fail(DGC_E_COLOR_CAP, "coloring move cap " + std::to_string(max_swaps) + " reached");
            }
            ++moves;
            if (nu > 0) {
                int64_t g = rng.choose(unv, nu);
                color[cur] = color[g];
                color[g] = -1;
                stamp[g] = chain;
                cur = g;
                ++s.swaps;
                continue;
            }
            unsigned both = uL & uR;
            if (both) {
                int n = C.list_of(both, buf);
                int8_t x = rng.choose(buf, n);
                int64_t gl = -1, gr = -1;
                for (int k = 0; k < F; ++k)
                    if (fl[k] >= 0 && color[fl[k]] == x) gl = fl[k];
                const int32_t *fr = &m.elem_face[rc * m.max_slots];
                for (int k = 0; k < F; ++k)
                    if (fr[k] >= 0 && color[fr[k]] == x) gr = fr[k];
                color[cur] = x;
                color[gl] = -1;
                color[gr] = -1;
                queue.push_back(gl);
                if (gr != gl) queue.push_back(gr);
                ++s.loop_breaks;
            } else {
                queue.push_back(cur);
                ++s.deferrals;
            }
            break;
        }
    }
    m.color.swap(color);
    m.n_colors = F;
    s.n_colors = F;
    for (int64_t f = 0; f < E; ++f) s.count[m.color[f]]++;
    if (st) *st = s;
    return DGC_OK;
}

dgc_status color_greedy_std(Mesh &m, dgc_color_stats *st) {
    const int64_t E = m.E;
    std::vector<int8_t> color(E, -1);
    Colorer C(m, color);
    int maxc = -1;
    for (int64_t f = 0; f < E; ++f) {
        unsigned u = C.used(m.face_L[f]) | C.used(m.face_R[f]);
        int c = 0;
        while (u & (1u << c)) ++c;
        if (c >= DGC_MAX_COLORS) return fail(DGC_E_UNSUPPORTED, "standard greedy needs more than 8 colors");
        color[f] = (int8_t)c;
        if (c > maxc) maxc = c;
    }
    m.color.swap(color);
    m.n_colors = maxc + 1;
    dgc_color_stats s{};
    s.n_colors = m.n_colors;
    for (int64_t f = 0; f < E; ++f) s.count[m.color[f]]++;
    if (st) *st = s;
    return DGC_OK;
}

bool coloring_valid(const Mesh &m, const std::vector<int8_t> &color, std::string *why) {
    if ((int64_t)color.size() != m.E) {
        if (why) *why = "coloring has the wrong length";
        return false;
    }
    for (int64_t f = 0; f < m.E; ++f) {
        if (color[f] < 0 || color[f] >= DGC_MAX_COLORS) {
            if (why) *why = "face " + std::to_string(f) + " has no valid color";
            return false;
        }
    }
    for (int64_t e = 0; e < m.K; ++e) {
        unsigned seen = 0;
        for (int k = 0; k < m.max_slots; ++k) {
            int32_t g = m.elem_face[e * m.max_slots + k];
            if (g < 0) continue;
            unsigned b = 1u << color[g];
            if (seen & b) {
                if (why) *why = "element " + std::to_string(e) + " has two faces of color " + std::to_string(color[g]);
                return false;
            }
            seen |= b;
        }
    }
    return true;
}

}  // namespace dgc
