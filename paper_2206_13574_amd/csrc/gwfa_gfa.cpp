// gwfa_gfa.cpp -- GFA 1 input: segments and links between oriented segments
// turned into the vertex-labelled directed graph of Definition 2.1.
//
// Each segment gives two vertices, its sequence (2i) and its reverse
// complement (2i+1); a link between oriented segments gives one edge and its
// complement (the same adjacency read on the other strand).  Host code only:
// nothing here touches a device.
#include <stdint.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <string>
#include <unordered_map>
#include <utility>
#include <vector>

#include "gwfa.h"

struct gwfa_gfa {
    bool forward = false;                  // GWFA_GFA_FORWARD: one vertex per segment
    std::vector<std::string> names;        // segment names in file order
    std::unordered_map<std::string, int32_t> index;
    std::string seq;                       // labels of all vertices, concatenated
    std::vector<int64_t> off;              // n_vtx + 1
    std::vector<std::pair<int32_t, int32_t>> edges;
    int64_t skipped = 0;                   // links dropped by GWFA_GFA_FORWARD
    int64_t err_line = 0;                  // 1-based line of the first error (0: none)
};

namespace {

inline bool acgt(char c) {
    const char u = (char)(c & 0xdf);
    return u == 'A' || u == 'C' || u == 'G' || u == 'T';
}

inline char complement(char c) {
    switch (c) {
    case 'A': return 'T';
    case 'C': return 'G';
    case 'G': return 'C';
    case 'T': return 'A';
    case 'a': return 't';
    case 'c': return 'g';
    case 'g': return 'c';
    default: return 'a';   // 't' (the alphabet is checked before)
    }
}

// Tab-separated fields of one line (no copies: views into the text).
struct Fields {
    const char* p[6];
    size_t n[6];
    int count = 0;
};

Fields split(const char* b, const char* e) {
    Fields f;
    const char* s = b;
    while (f.count < 6) {
        const char* t = static_cast<const char*>(memchr(s, '\t', (size_t)(e - s)));
        const char* end = t ? t : e;
        f.p[f.count] = s;
        f.n[f.count] = (size_t)(end - s);
        ++f.count;
        if (!t) break;
        s = t + 1;
    }
    return f;
}

bool is_orient(const char* p, size_t n) { return n == 1 && (p[0] == '+' || p[0] == '-'); }

// An overlap the graph model can hold: none ("*", or a CIGAR of zero-length
// match such as "0M").
bool zero_overlap(const char* p, size_t n) {
    if (n == 1 && p[0] == '*') return true;
    if (n < 2 || p[n - 1] != 'M') return false;
    for (size_t i = 0; i + 1 < n; ++i)
        if (p[i] != '0') return false;
    return true;
}

int parse(const char* text, int64_t len, int32_t flags, gwfa_gfa* g) {
    g->forward = (flags & GWFA_GFA_FORWARD) != 0;
    const char* end = text + len;
    // pass 1: segments; pass 2: links (links may name segments defined later)
    for (int pass = 0; pass < 2; ++pass) {
        int64_t line = 0;
        for (const char* b = text; b < end;) {
            const char* nl = static_cast<const char*>(memchr(b, '\n', (size_t)(end - b)));
            const char* e = nl ? nl : end;
            const char* next = nl ? nl + 1 : end;
            ++line;
            if (e > b && e[-1] == '\r') --e;
            if (e == b || (pass == 0 && *b != 'S') || (pass == 1 && *b != 'L')) { b = next; continue; }
            const Fields f = split(b, e);
            if (f.n[0] != 1) { b = next; continue; }   // another record type starting with S or L
            if (pass == 0) {
                if (f.count < 3 || f.n[1] == 0) { g->err_line = line; return GWFA_ERR_FORMAT; }
                std::string name(f.p[1], f.n[1]);
                if (g->index.count(name)) { g->err_line = line; return GWFA_ERR_FORMAT; }
                if (f.n[2] == 1 && f.p[2][0] == '*') { g->err_line = line; return GWFA_ERR_UNSUPPORTED; }
                if (f.n[2] == 0) { g->err_line = line; return GWFA_ERR_EMPTY_LABEL; }
                for (size_t i = 0; i < f.n[2]; ++i)
                    if (!acgt(f.p[2][i])) { g->err_line = line; return GWFA_ERR_ALPHABET; }
                const int32_t id = (int32_t)g->names.size();
                if (id >= (g->forward ? INT32_MAX : INT32_MAX / 2)) { g->err_line = line; return GWFA_ERR_ARG; }
                g->index.emplace(name, id);
                g->names.push_back(std::move(name));
                if (g->off.empty()) g->off.push_back(0);
                g->seq.append(f.p[2], f.n[2]);
                g->off.push_back((int64_t)g->seq.size());
                if (!g->forward) {
                    for (size_t i = f.n[2]; i-- > 0;) g->seq.push_back(complement(f.p[2][i]));
                    g->off.push_back((int64_t)g->seq.size());
                }
            } else {
                if (f.count < 6 || !is_orient(f.p[2], f.n[2]) || !is_orient(f.p[4], f.n[4])) {
                    g->err_line = line;
                    return GWFA_ERR_FORMAT;
                }
                if (!zero_overlap(f.p[5], f.n[5])) { g->err_line = line; return GWFA_ERR_UNSUPPORTED; }
                const auto a = g->index.find(std::string(f.p[1], f.n[1]));
                const auto c = g->index.find(std::string(f.p[3], f.n[3]));
                if (a == g->index.end() || c == g->index.end()) { g->err_line = line; return GWFA_ERR_VERTEX; }
                const int ra = f.p[2][0] == '-', rc = f.p[4][0] == '-';
                if (g->forward) {
                    if (ra || rc) { ++g->skipped; b = next; continue; }
                    g->edges.emplace_back(a->second, c->second);
                } else {
                    const int32_t u = 2 * a->second + ra, w = 2 * c->second + rc;
                    g->edges.emplace_back(u, w);
                    g->edges.emplace_back(w ^ 1, u ^ 1);   // the same link on the other strand
                }
            }
            b = next;
        }
    }
    if (g->names.empty()) { g->err_line = 0; return GWFA_ERR_FORMAT; }
    std::sort(g->edges.begin(), g->edges.end());
    g->edges.erase(std::unique(g->edges.begin(), g->edges.end()), g->edges.end());
    return GWFA_OK;
}

}  // namespace

extern "C" {

int gwfa_gfa_parse(const char* text, int64_t len, int32_t flags, gwfa_gfa** out, int64_t* err_line) {
    if (err_line) *err_line = 0;
    if (!out || (len > 0 && !text) || len < 0 || (flags & ~GWFA_GFA_FORWARD)) return GWFA_ERR_ARG;
    *out = nullptr;
    gwfa_gfa* g = new (std::nothrow) gwfa_gfa();
    if (!g) return GWFA_ERR_NOMEM;
    int rc;
    try {
        rc = parse(text, len, flags, g);
    } catch (...) {
        rc = GWFA_ERR_NOMEM;
    }
    if (rc != GWFA_OK) {
        if (err_line) *err_line = g->err_line;
        delete g;
        return rc;
    }
    *out = g;
    return GWFA_OK;
}

int gwfa_gfa_load(const char* path, int32_t flags, gwfa_gfa** out, int64_t* err_line) {
    if (err_line) *err_line = 0;
    if (!path || !out) return GWFA_ERR_ARG;
    *out = nullptr;
    FILE* fp = fopen(path, "rb");
    if (!fp) return GWFA_ERR_ARG;
    std::string text;
    char buf[1 << 16];
    size_t n;
    try {
        while ((n = fread(buf, 1, sizeof(buf), fp)) > 0) text.append(buf, n);
    } catch (...) {
        fclose(fp);
        return GWFA_ERR_NOMEM;
    }
    const bool bad = ferror(fp) != 0;
    fclose(fp);
    if (bad) return GWFA_ERR_ARG;
    return gwfa_gfa_parse(text.data(), (int64_t)text.size(), flags, out, err_line);
}

int gwfa_gfa_sizes(const gwfa_gfa* g, int32_t* n_vtx, int64_t* n_bases, int64_t* n_edge, int32_t* n_segments,
                   int64_t* n_skipped) {
    if (!g) return GWFA_ERR_ARG;
    if (n_vtx) *n_vtx = (int32_t)(g->off.size() - 1);
    if (n_bases) *n_bases = (int64_t)g->seq.size();
    if (n_edge) *n_edge = (int64_t)g->edges.size();
    if (n_segments) *n_segments = (int32_t)g->names.size();
    if (n_skipped) *n_skipped = g->skipped;
    return GWFA_OK;
}

int gwfa_gfa_graph(const gwfa_gfa* g, uint8_t* seq, int64_t* seq_off, int32_t* edge_src, int32_t* edge_dst) {
    if (!g || !seq || !seq_off || (!g->edges.empty() && (!edge_src || !edge_dst))) return GWFA_ERR_ARG;
    memcpy(seq, g->seq.data(), g->seq.size());
    memcpy(seq_off, g->off.data(), g->off.size() * sizeof(int64_t));
    for (size_t e = 0; e < g->edges.size(); ++e) {
        edge_src[e] = g->edges[e].first;
        edge_dst[e] = g->edges[e].second;
    }
    return GWFA_OK;
}

int32_t gwfa_gfa_vertex(const gwfa_gfa* g, const char* name, int32_t reverse) {
    if (!g || !name || (reverse != 0 && reverse != 1)) return GWFA_ERR_ARG;
    const auto it = g->index.find(name);
    if (it == g->index.end() || (g->forward && reverse)) return GWFA_ERR_VERTEX;
    return g->forward ? it->second : 2 * it->second + reverse;
}

const char* gwfa_gfa_name(const gwfa_gfa* g, int32_t v, int32_t* reverse) {
    if (!g || v < 0 || v >= (int32_t)(g->off.size() - 1)) return nullptr;
    if (reverse) *reverse = g->forward ? 0 : (v & 1);
    return g->names[(size_t)(g->forward ? v : v >> 1)].c_str();
}

void gwfa_gfa_free(gwfa_gfa* g) { delete g; }

}  // extern "C"
