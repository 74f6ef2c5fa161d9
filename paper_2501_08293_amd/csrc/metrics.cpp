// Per-solve metrics records: when the environment variable OPF_ADMM_METRICS
// names a file, every single-instance solve, batched solve and served request
// appends one JSON object as a line of it (JSON Lines): sizes, schedule,
// status, iterations, residuals, times, iteration rate and the effective
// bandwidth of the algorithmic bytes.  Writes from several threads are
// serialised; failing to open the file drops the record.
#include "metrics.h"

#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <mutex>

namespace opf {
namespace {
std::mutex g_metrics_mu;

std::string number(double v) {
    if (!std::isfinite(v)) return "null";
    char buf[40];
    std::snprintf(buf, sizeof(buf), "%.17g", v);
    return buf;
}
}  // namespace

void JsonLine::key(const char* k) {
    if (!body_.empty()) body_ += ", ";
    body_ += '"';
    body_ += k;
    body_ += "\": ";
}

JsonLine& JsonLine::str(const char* k, const std::string& v) {
    key(k);
    body_ += '"';
    for (char c : v) {
        if (c == '"' || c == '\\') body_ += '\\';
        body_ += c;
    }
    body_ += '"';
    return *this;
}

JsonLine& JsonLine::num(const char* k, double v) {
    key(k);
    body_ += number(v);
    return *this;
}

JsonLine& JsonLine::integer(const char* k, long long v) {
    key(k);
    body_ += std::to_string(v);
    return *this;
}

JsonLine& JsonLine::pairs(const char* k, const std::vector<std::pair<double, double>>& v) {
    key(k);
    body_ += '[';
    for (size_t i = 0; i < v.size(); ++i) {
        if (i) body_ += ", ";
        body_ += "[" + number(v[i].first) + ", " + number(v[i].second) + "]";
    }
    body_ += ']';
    return *this;
}

bool metrics_on() {
    const char* p = std::getenv("OPF_ADMM_METRICS");
    return p && *p;
}

void metrics_write(const JsonLine& line) {
    const char* p = std::getenv("OPF_ADMM_METRICS");
    if (!p || !*p) return;
    const std::string t = line.text() + "\n";
    std::lock_guard<std::mutex> lk(g_metrics_mu);
    if (FILE* f = std::fopen(p, "a")) {
        std::fwrite(t.data(), 1, t.size(), f);
        std::fclose(f);
    }
}

}  // namespace opf
