// Launch-parameter table of the autotuner.  Entries are keyed by a graph
// signature; they change only speed (chunk sizes, persistent grid size) and,
// for the heavy multiplier, the reported light/heavy split, never the count.
#include "tc_internal.h"

#include <map>
#include <mutex>
#include <tuple>

namespace tc {

namespace {
std::mutex g_tune_mu;
// (n, m, sampled, p in millionths) -> config
std::map<std::tuple<int64_t, int64_t, int, int64_t>, CountConfig> g_table;

std::tuple<int64_t, int64_t, int, int64_t> key_of(const tc_graph_s* g, int sampled, double p) {
    return std::make_tuple(g->n, g->m, sampled, (int64_t)(p * 1e6 + 0.5));
}
}  // namespace

CountConfig tuned_config(const tc_graph_s* g, int sampled, double p, const CountConfig& base) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    auto it = g_table.find(key_of(g, sampled, p));
    return it == g_table.end() ? base : it->second;
}

void tune_store(const tc_graph_s* g, int sampled, double p, const CountConfig& c) {
    std::lock_guard<std::mutex> lk(g_tune_mu);
    g_table[key_of(g, sampled, p)] = c;
}

}  // namespace tc
