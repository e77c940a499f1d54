// Reading and writing bundle-adjustment problems in the BAL text format, the
// format of the Bundle Adjustment in the Large datasets the paper evaluates on
// (Section VI).  Host code only.
//
// A BAL file is a stream of whitespace-separated tokens:
//   n_cams n_points n_obs
//   n_obs records      camera point x y       (integer, integer, real, real)
//   n_cams records     9 reals: angle-axis rotation, translation, f, k1, k2
//   n_points records   3 reals
// The reader tokenises the file in parallel: every thread counts the tokens
// of its byte range (cut at whitespace), a prefix sum gives each range the
// index of its first token, and the token index alone decides which array
// slot a token fills.  Reals are parsed with std::from_chars (correctly
// rounded), so a file written with round-trip precision reads back exactly.
#include <algorithm>
#include <charconv>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <string>
#include <thread>
#include <vector>

#include "common.hpp"

namespace cba {
namespace {

inline bool is_space(char c) { return c == ' ' || c == '\n' || c == '\r' || c == '\t' || c == '\v' || c == '\f'; }

struct FileBuf {
  std::vector<char> data;
};

FileBuf read_file(const char* path) {
  if (path == nullptr) fail(CASPAR_EINVAL, "BAL: null path");
  FILE* f = std::fopen(path, "rb");
  if (!f) fail(CASPAR_EIO, std::string("BAL: cannot open ") + path);
  FileBuf b;
  if (std::fseek(f, 0, SEEK_END) != 0) {
    std::fclose(f);
    fail(CASPAR_EIO, std::string("BAL: cannot seek ") + path);
  }
  const long n = std::ftell(f);
  std::rewind(f);
  if (n < 0) {
    std::fclose(f);
    fail(CASPAR_EIO, std::string("BAL: cannot size ") + path);
  }
  b.data.resize((size_t)n);
  const size_t got = n > 0 ? std::fread(b.data.data(), 1, (size_t)n, f) : 0;
  std::fclose(f);
  if (got != (size_t)n) fail(CASPAR_EIO, std::string("BAL: short read of ") + path);
  return b;
}

// Next token in [p, end): returns false at the end of the range.
inline bool next_token(const char*& p, const char* end, const char*& tb, const char*& te) {
  while (p < end && is_space(*p)) ++p;
  if (p >= end) return false;
  tb = p;
  while (p < end && !is_space(*p)) ++p;
  te = p;
  return true;
}

inline bool parse_int(const char* tb, const char* te, long long& v) {
  if (tb < te && *tb == '+') ++tb;
  const auto r = std::from_chars(tb, te, v);
  return r.ec == std::errc() && r.ptr == te;
}

inline bool parse_real(const char* tb, const char* te, double& v) {
  if (tb < te && *tb == '+') ++tb;
  const auto r = std::from_chars(tb, te, v, std::chars_format::general);
  return r.ec == std::errc() && r.ptr == te && std::isfinite(v);
}

std::string token_text(const char* tb, const char* te) {
  return std::string(tb, (size_t)std::min<ptrdiff_t>(te - tb, 40));
}

struct Header {
  long long nc, np, no;
  const char* body;  // first byte after the header
};

Header parse_header(const FileBuf& b) {
  const char* p = b.data.data();
  const char* end = p + b.data.size();
  long long v[3];
  for (int i = 0; i < 3; ++i) {
    const char *tb, *te;
    if (!next_token(p, end, tb, te)) fail(CASPAR_EINVAL, "BAL: file ends inside the header");
    if (!parse_int(tb, te, v[i]) || v[i] < 0)
      fail(CASPAR_EINVAL, "BAL: header count '" + token_text(tb, te) + "' is not a non-negative integer");
  }
  if (v[0] > INT32_MAX || v[1] > INT32_MAX) fail(CASPAR_EINVAL, "BAL: camera or point count exceeds int32");
  if (v[2] > (1LL << 40)) fail(CASPAR_EINVAL, "BAL: observation count exceeds 2^40");
  return Header{v[0], v[1], v[2], p};
}

struct Outputs {
  int32_t* obs_cam;
  int32_t* obs_pt;
  double* px;
  double* cams;
  double* points;
};

// Token k of the body (after the header) goes to one slot of the outputs.
struct Fill {
  long long nc, np, no;
  Outputs o;
  // returns an error message, empty when the token was stored
  std::string operator()(long long k, const char* tb, const char* te) const {
    const long long n_obs_tok = 4 * no;
    if (k < n_obs_tok) {
      const long long i = k / 4;
      const int f = (int)(k % 4);
      if (f < 2) {
        long long v;
        if (!parse_int(tb, te, v)) return "observation " + std::to_string(i) + ": index '" + token_text(tb, te) + "' is not an integer";
        const long long lim = f == 0 ? nc : np;
        if (v < 0 || v >= lim)
          return "observation " + std::to_string(i) + ": " + (f == 0 ? "camera" : "point") + " index " +
                 std::to_string(v) + " out of range";
        (f == 0 ? o.obs_cam : o.obs_pt)[i] = (int32_t)v;
      } else {
        double v;
        if (!parse_real(tb, te, v)) return "observation " + std::to_string(i) + ": pixel '" + token_text(tb, te) + "' is not a finite number";
        o.px[2 * i + (f - 2)] = v;
      }
      return {};
    }
    k -= n_obs_tok;
    double v;
    if (k < 9 * nc) {
      if (!parse_real(tb, te, v)) return "camera " + std::to_string(k / 9) + ": '" + token_text(tb, te) + "' is not a finite number";
      o.cams[k] = v;
      return {};
    }
    k -= 9 * nc;
    if (k < 3 * np) {
      if (!parse_real(tb, te, v)) return "point " + std::to_string(k / 3) + ": '" + token_text(tb, te) + "' is not a finite number";
      o.points[k] = v;
      return {};
    }
    return "trailing data after the last point";
  }
};

void parse_body(const FileBuf& b, const Header& h, const Outputs& out) {
  const char* body = h.body;
  const char* end = b.data.data() + b.data.size();
  const long long want = 4 * h.no + 9 * h.nc + 3 * h.np;
  const size_t bytes = (size_t)(end - body);
  const unsigned hw = std::max(1u, std::thread::hardware_concurrency());
  const int T = (int)std::min<size_t>(std::min(hw, 16u), std::max<size_t>(1, bytes / (1u << 20)));
  // byte ranges cut at whitespace so that no token straddles two ranges
  std::vector<const char*> cut(T + 1);
  cut[0] = body;
  cut[T] = end;
  for (int t = 1; t < T; ++t) {
    const char* c = body + bytes * t / T;
    c = std::max(c, cut[t - 1]);
    while (c < end && !is_space(*c)) ++c;
    cut[t] = c;
  }
  std::vector<long long> count(T, 0);
  auto count_range = [&](int t) {
    const char* p = cut[t];
    const char *tb, *te;
    long long n = 0;
    while (next_token(p, cut[t + 1], tb, te)) ++n;
    count[t] = n;
  };
  {
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(count_range, t);
    count_range(0);
    for (auto& x : th) x.join();
  }
  long long total = 0;
  std::vector<long long> first(T);
  for (int t = 0; t < T; ++t) {
    first[t] = total;
    total += count[t];
  }
  if (total < want)
    fail(CASPAR_EINVAL, "BAL: file ends early: " + std::to_string(total) + " values after the header, " +
                            std::to_string(want) + " expected");
  if (total > want) fail(CASPAR_EINVAL, "BAL: trailing data after the last point");
  const Fill fill{h.nc, h.np, h.no, out};
  // first error of each range; the earliest range's error is reported
  std::vector<std::string> err(T);
  auto fill_range = [&](int t) {
    const char* p = cut[t];
    const char *tb, *te;
    long long k = first[t];
    while (next_token(p, cut[t + 1], tb, te)) {
      std::string e = fill(k++, tb, te);
      if (!e.empty()) {
        err[t] = std::move(e);
        return;
      }
    }
  };
  {
    std::vector<std::thread> th;
    for (int t = 1; t < T; ++t) th.emplace_back(fill_range, t);
    fill_range(0);
    for (auto& x : th) x.join();
  }
  for (int t = 0; t < T; ++t)
    if (!err[t].empty()) fail(CASPAR_EINVAL, "BAL: " + err[t]);
}

void put(std::string& s, double v) {
  char buf[32];
  const auto r = std::to_chars(buf, buf + sizeof(buf), v);  // shortest round-trip form
  s.append(buf, r.ptr);
}

}  // namespace
}  // namespace cba

using namespace cba;

#define CBA_API_BEGIN try {
#define CBA_API_END                  \
  }                                  \
  catch (const Error& e) {           \
    set_last_error(e.msg);           \
    return e.status;                 \
  }                                  \
  catch (const std::exception& e) {  \
    set_last_error(e.what());        \
    return CASPAR_EIO;               \
  }                                  \
  set_last_error("");                \
  return CASPAR_OK;

extern "C" {

int caspar_bal_read_header(const char* path, int32_t* n_cams, int32_t* n_points, int64_t* n_obs) {
  CBA_API_BEGIN
  const FileBuf b = read_file(path);
  const Header h = parse_header(b);
  if (n_cams) *n_cams = (int32_t)h.nc;
  if (n_points) *n_points = (int32_t)h.np;
  if (n_obs) *n_obs = (int64_t)h.no;
  CBA_API_END
}

int caspar_bal_read(const char* path, int32_t n_cams, int32_t n_points, int64_t n_obs, int32_t* obs_cam,
                    int32_t* obs_pt, double* px, double* cams, double* points) {
  CBA_API_BEGIN
  const FileBuf b = read_file(path);
  const Header h = parse_header(b);
  if (h.nc != n_cams || h.np != n_points || h.no != n_obs)
    fail(CASPAR_EINVAL, "BAL: sizes passed (" + std::to_string(n_cams) + ", " + std::to_string(n_points) + ", " +
                            std::to_string(n_obs) + ") differ from the file's header (" + std::to_string(h.nc) +
                            ", " + std::to_string(h.np) + ", " + std::to_string(h.no) + ")");
  if ((n_obs > 0 && (!obs_cam || !obs_pt || !px)) || (n_cams > 0 && !cams) || (n_points > 0 && !points))
    fail(CASPAR_EINVAL, "BAL: null output array");
  parse_body(b, h, Outputs{obs_cam, obs_pt, px, cams, points});
  CBA_API_END
}

int caspar_bal_write(const char* path, int32_t n_cams, int32_t n_points, int64_t n_obs, const int32_t* obs_cam,
                     const int32_t* obs_pt, const double* px, const double* cams, const double* points) {
  CBA_API_BEGIN
  if (path == nullptr) fail(CASPAR_EINVAL, "BAL: null path");
  if (n_cams < 0 || n_points < 0 || n_obs < 0) fail(CASPAR_EINVAL, "BAL: negative size");
  if ((n_obs > 0 && (!obs_cam || !obs_pt || !px)) || (n_cams > 0 && !cams) || (n_points > 0 && !points))
    fail(CASPAR_EINVAL, "BAL: null input array");
  for (int64_t i = 0; i < n_obs; ++i) {
    if (obs_cam[i] < 0 || obs_cam[i] >= n_cams || obs_pt[i] < 0 || obs_pt[i] >= n_points)
      fail(CASPAR_EINVAL, "BAL: observation " + std::to_string(i) + " has an index out of range");
    if (!std::isfinite(px[2 * i]) || !std::isfinite(px[2 * i + 1]))
      fail(CASPAR_EINVAL, "BAL: observation " + std::to_string(i) + " has a non-finite pixel");
  }
  for (int64_t k = 0; k < 9 * (int64_t)n_cams; ++k)
    if (!std::isfinite(cams[k])) fail(CASPAR_EINVAL, "BAL: camera " + std::to_string(k / 9) + " has a non-finite value");
  for (int64_t k = 0; k < 3 * (int64_t)n_points; ++k)
    if (!std::isfinite(points[k])) fail(CASPAR_EINVAL, "BAL: point " + std::to_string(k / 3) + " has a non-finite value");
  FILE* f = std::fopen(path, "wb");
  if (!f) fail(CASPAR_EIO, std::string("BAL: cannot create ") + path);
  std::string s;
  s.reserve(1 << 22);
  auto flush = [&](bool force) {
    if (s.size() >= (1u << 22) || (force && !s.empty())) {
      const size_t w = std::fwrite(s.data(), 1, s.size(), f);
      const bool ok = w == s.size();
      s.clear();
      if (!ok) {
        std::fclose(f);
        fail(CASPAR_EIO, std::string("BAL: short write to ") + path);
      }
    }
  };
  s += std::to_string(n_cams) + " " + std::to_string(n_points) + " " + std::to_string(n_obs) + "\n";
  for (int64_t i = 0; i < n_obs; ++i) {
    s += std::to_string(obs_cam[i]);
    s += ' ';
    s += std::to_string(obs_pt[i]);
    s += ' ';
    put(s, px[2 * i]);
    s += ' ';
    put(s, px[2 * i + 1]);
    s += '\n';
    flush(false);
  }
  for (int64_t k = 0; k < 9 * (int64_t)n_cams; ++k) {
    put(s, cams[k]);
    s += '\n';
    flush(false);
  }
  for (int64_t k = 0; k < 3 * (int64_t)n_points; ++k) {
    put(s, points[k]);
    s += '\n';
    flush(false);
  }
  flush(true);
  if (std::fclose(f) != 0) fail(CASPAR_EIO, std::string("BAL: cannot close ") + path);
  CBA_API_END
}

}  // extern "C"
