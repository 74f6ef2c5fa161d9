// Per-solve metrics records (internal header; see metrics.cpp).
#pragma once

#include <string>
#include <utility>
#include <vector>

namespace opf {

// One JSON object built field by field; non-finite numbers become null.
class JsonLine {
public:
    JsonLine& str(const char* k, const std::string& v);
    JsonLine& num(const char* k, double v);
    JsonLine& integer(const char* k, long long v);
    JsonLine& pairs(const char* k, const std::vector<std::pair<double, double>>& v);
    std::string text() const { return "{" + body_ + "}"; }

private:
    void key(const char* k);
    std::string body_;
};

// Whether records are wanted (the environment variable OPF_ADMM_METRICS names
// a file), and appending one record as a line of that file.
bool metrics_on();
void metrics_write(const JsonLine& line);

}  // namespace opf
