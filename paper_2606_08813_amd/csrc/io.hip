// An index as a directory of files (the immutable segment of Section 2 and
// Fig. 1, on disk): NumPy .npy arrays in the stored format plus meta.json with
// the sizes and a 64-bit FNV-1a checksum (Fowler, Noll and Vo) of every file's
// data bytes.  The .npy files follow NumPy's format 1.0 (magic, version,
// little-endian header length, a Python-literal header dict padded to a
// multiple of 64 bytes, then C-order data), so numpy.load reads them directly.
#include <cstdio>
#include <cstring>
#include <filesystem>
#include <fstream>
#include <sstream>
#include <string>
#include <vector>

#include "hntl_internal.h"

namespace fs = std::filesystem;

namespace hntl {
namespace {

struct IoError {
  std::string msg;
};

constexpr uint64_t FNV_OFFSET = 1469598103934665603ull, FNV_PRIME = 1099511628211ull;
void fnv1a(uint64_t& h, const void* p, size_t n) {
  const unsigned char* c = static_cast<const unsigned char*>(p);
  for (size_t i = 0; i < n; ++i) {
    h ^= c[i];
    h *= FNV_PRIME;
  }
}
std::string hex64(uint64_t h) {
  char b[17];
  std::snprintf(b, sizeof(b), "%016llx", (unsigned long long)h);
  return b;
}

std::string shape_str(const std::vector<int64_t>& shape) {
  std::string s = "(";
  for (size_t i = 0; i < shape.size(); ++i) s += std::to_string(shape[i]) + (shape.size() == 1 || i + 1 < shape.size() ? ", " : "");
  if (shape.size() == 1) s.pop_back();
  return s + ")";
}

// Writes one .npy file whose data comes from `fill` in pieces (fill(offset,
// bytes, dst) copies that byte range); returns the checksum of the data.
template <class Fill>
std::string write_npy(const fs::path& p, const char* descr, const std::vector<int64_t>& shape, size_t bytes,
                      Fill fill) {
  std::string dict = std::string("{'descr': '") + descr + "', 'fortran_order': False, 'shape': " + shape_str(shape) +
                     ", }";
  size_t hl = dict.size() + 1;  // + '\n'
  while ((10 + hl) % 64 != 0) ++hl;
  dict.append(hl - 1 - dict.size(), ' ');
  dict += '\n';
  std::ofstream f(p, std::ios::binary | std::ios::trunc);
  if (!f) throw IoError{"cannot write " + p.string()};
  const char magic[8] = {'\x93', 'N', 'U', 'M', 'P', 'Y', 1, 0};
  f.write(magic, 8);
  const uint16_t len = (uint16_t)hl;
  const unsigned char lb[2] = {(unsigned char)(len & 0xff), (unsigned char)(len >> 8)};
  f.write(reinterpret_cast<const char*>(lb), 2);
  f.write(dict.data(), (std::streamsize)dict.size());
  uint64_t h = FNV_OFFSET;
  const size_t piece = (size_t)256 << 20;
  std::vector<char> buf(std::min(bytes, piece));
  for (size_t off = 0; off < bytes; off += piece) {
    const size_t n = std::min(piece, bytes - off);
    fill(off, n, buf.data());
    fnv1a(h, buf.data(), n);
    f.write(buf.data(), (std::streamsize)n);
  }
  if (!f) throw IoError{"write failed: " + p.string()};
  return hex64(h);
}

struct NpyReader {
  std::ifstream f;
  std::vector<int64_t> shape;
  std::string descr;
  size_t bytes = 0;
  uint64_t h = FNV_OFFSET;

  NpyReader(const fs::path& p, const char* want_descr) : f(p, std::ios::binary) {
    if (!f) throw IoError{"cannot read " + p.string()};
    char magic[8];
    f.read(magic, 8);
    if (!f || std::memcmp(magic, "\x93NUMPY", 6) != 0) throw IoError{"not a .npy file: " + p.string()};
    size_t hl = 0;
    if (magic[6] == 1) {
      unsigned char lb[2];
      f.read(reinterpret_cast<char*>(lb), 2);
      hl = lb[0] | (lb[1] << 8);
    } else if (magic[6] == 2 || magic[6] == 3) {
      unsigned char lb[4];
      f.read(reinterpret_cast<char*>(lb), 4);
      hl = lb[0] | (lb[1] << 8) | ((size_t)lb[2] << 16) | ((size_t)lb[3] << 24);
    } else {
      throw IoError{"unknown .npy version: " + p.string()};
    }
    std::string dict(hl, '\0');
    f.read(&dict[0], (std::streamsize)hl);
    if (!f) throw IoError{"truncated header: " + p.string()};
    auto field = [&](const char* key) -> std::string {
      const size_t k = dict.find(std::string("'") + key + "'");
      if (k == std::string::npos) throw IoError{std::string("header lacks ") + key + ": " + p.string()};
      return dict.substr(dict.find(':', k) + 1);
    };
    std::string d = field("descr");
    const size_t q0 = d.find('\''), q1 = d.find('\'', q0 + 1);
    descr = d.substr(q0 + 1, q1 - q0 - 1);
    if (descr != want_descr) throw IoError{"dtype " + descr + " where " + want_descr + " was expected: " + p.string()};
    if (field("fortran_order").find("False") > 2) throw IoError{"Fortran-order array: " + p.string()};
    std::string sh = field("shape");
    sh = sh.substr(sh.find('(') + 1, sh.find(')') - sh.find('(') - 1);
    std::stringstream ss(sh);
    std::string tok;
    while (std::getline(ss, tok, ','))
      if (tok.find_first_not_of(" ") != std::string::npos) shape.push_back(std::stoll(tok));
    size_t el = 1;
    for (int64_t s : shape) el *= (size_t)s;
    bytes = el * (descr[2] - '0');
  }
  // Reads the next n data bytes into dst, checksumming them.
  void read(void* dst, size_t n) {
    f.read(static_cast<char*>(dst), (std::streamsize)n);
    if (!f) throw IoError{"truncated data"};
    fnv1a(h, dst, n);
  }
};

std::string json_str(const std::string& js, const std::string& key) {
  const size_t k = js.find("\"" + key + "\"");
  if (k == std::string::npos) return "";
  const size_t c = js.find(':', k);
  const size_t a = js.find_first_not_of(" \t\n", c + 1);
  if (js[a] == '"') return js.substr(a + 1, js.find('"', a + 1) - a - 1);
  const size_t b = js.find_first_of(",}\n", a);
  return js.substr(a, b - a);
}
int64_t json_int(const std::string& js, const std::string& key) {
  const std::string v = json_str(js, key);
  if (v.empty()) throw IoError{"meta.json lacks " + key};
  return std::stoll(v);
}

void expect_shape(const NpyReader& r, const std::vector<int64_t>& want, const char* name) {
  if (r.shape != want) throw IoError{std::string(name) + " has shape " + shape_str(r.shape) + ", expected " + shape_str(want)};
}

template <class T>
std::vector<T> read_all(const fs::path& dir, const char* name, const char* descr, const std::vector<int64_t>& shape,
                        const std::string& meta) {
  NpyReader r(dir / name, descr);
  expect_shape(r, shape, name);
  std::vector<T> v(r.bytes / sizeof(T));
  r.read(v.data(), r.bytes);
  if (hex64(r.h) != json_str(meta, name)) throw IoError{std::string("checksum mismatch: ") + name};
  return v;
}

}  // namespace
}  // namespace hntl

using namespace hntl;

extern "C" hntl_status hntl_index_save(const hntl_index* index, const char* dir) {
  set_error("");
  if (!index || !dir) return fail(HNTL_EINVAL, "null pointer");
  const Index& ix = index->ix;
  try {
    HIP_TRY(hipSetDevice(ix.device));
    HIP_TRY(hipDeviceSynchronize());
    const fs::path p(dir);
    std::error_code ec;
    fs::create_directories(p, ec);
    if (!fs::is_directory(p)) throw IoError{"cannot create directory " + p.string()};
    const int64_t N = (int64_t)ix.N, d = ix.d, G = ix.G, r = ix.r;
    std::vector<float> cen((size_t)G * d), bas((size_t)G * r * d), codes((size_t)N * r), eps(N);
    std::vector<int64_t> off(G + 1);
    std::vector<int32_t> perm(N);
    const hntl_status st =
        hntl_index_export(index, cen.data(), bas.data(), off.data(), perm.data(), codes.data(), eps.data(), nullptr);
    if (st != HNTL_OK) return st;
    std::vector<std::pair<std::string, std::string>> sums;
    auto host = [](const void* src) {
      return [src](size_t o, size_t n, char* dst) { std::memcpy(dst, static_cast<const char*>(src) + o, n); };
    };
    sums.emplace_back("centroids.npy", write_npy(p / "centroids.npy", "<f4", {G, d}, cen.size() * 4, host(cen.data())));
    sums.emplace_back("basis.npy", write_npy(p / "basis.npy", "<f4", {G, r, d}, bas.size() * 4, host(bas.data())));
    sums.emplace_back("offsets.npy", write_npy(p / "offsets.npy", "<i8", {G + 1}, off.size() * 8, host(off.data())));
    sums.emplace_back("perm.npy", write_npy(p / "perm.npy", "<i4", {N}, perm.size() * 4, host(perm.data())));
    sums.emplace_back("codes.npy", write_npy(p / "codes.npy", "<f4", {N, r}, codes.size() * 4, host(codes.data())));
    sums.emplace_back("eps.npy", write_npy(p / "eps.npy", "<f4", {N}, eps.size() * 4, host(eps.data())));
    if (ix.X) {  // raw vectors streamed from the device in pieces
      const float* X = ix.X;
      sums.emplace_back("X.npy", write_npy(p / "X.npy", "<f4", {N, d}, (size_t)N * d * 4, [X](size_t o, size_t n, char* dst) {
                          HIP_TRY(hipMemcpy(dst, reinterpret_cast<const char*>(X) + o, n, hipMemcpyDeviceToHost));
                        }));
    }
    bool have_cap = ix.captured.size() == ix.G;
    if (have_cap) {
      have_cap = false;
      for (double c : ix.captured) have_cap = have_cap || c >= 0.0;
    }
    if (have_cap)
      sums.emplace_back("captured.npy", write_npy(p / "captured.npy", "<f8", {G}, (size_t)G * 8, host(ix.captured.data())));
    uint32_t h1 = 0, h2 = 0;
    if (ix.router) {
      h1 = (uint32_t)ix.router->h1;
      h2 = (uint32_t)ix.router->h2;
      std::vector<float> W1((size_t)h1 * d), b1(h1), W2((size_t)h2 * h1), b2(h2), W3((size_t)G * h2), b3(G), mu(d), sd(d);
      const hntl_status rs = hntl_router_export(index, nullptr, nullptr, W1.data(), b1.data(), W2.data(), b2.data(),
                                                W3.data(), b3.data(), mu.data(), sd.data());
      if (rs != HNTL_OK) return rs;
      const int64_t H1 = h1, H2 = h2;
      sums.emplace_back("router_W1.npy", write_npy(p / "router_W1.npy", "<f4", {H1, d}, W1.size() * 4, host(W1.data())));
      sums.emplace_back("router_b1.npy", write_npy(p / "router_b1.npy", "<f4", {H1}, b1.size() * 4, host(b1.data())));
      sums.emplace_back("router_W2.npy", write_npy(p / "router_W2.npy", "<f4", {H2, H1}, W2.size() * 4, host(W2.data())));
      sums.emplace_back("router_b2.npy", write_npy(p / "router_b2.npy", "<f4", {H2}, b2.size() * 4, host(b2.data())));
      sums.emplace_back("router_W3.npy", write_npy(p / "router_W3.npy", "<f4", {G, H2}, W3.size() * 4, host(W3.data())));
      sums.emplace_back("router_b3.npy", write_npy(p / "router_b3.npy", "<f4", {G}, b3.size() * 4, host(b3.data())));
      sums.emplace_back("router_mean.npy", write_npy(p / "router_mean.npy", "<f4", {d}, mu.size() * 4, host(mu.data())));
      sums.emplace_back("router_std.npy", write_npy(p / "router_std.npy", "<f4", {d}, sd.size() * 4, host(sd.data())));
    }
    std::ofstream m(p / "meta.json", std::ios::trunc);
    if (!m) throw IoError{"cannot write meta.json"};
    m << "{\n  \"format\": \"hntl-index\",\n  \"version\": 1,\n  \"N\": " << N << ",\n  \"d\": " << d
      << ",\n  \"G\": " << G << ",\n  \"r\": " << r << ",\n  \"codes_mask\": " << ix.codes_mask
      << ",\n  \"raw_vectors\": " << (ix.X ? 1 : 0) << ",\n  \"captured\": " << (have_cap ? 1 : 0)
      << ",\n  \"router_hidden1\": " << h1 << ",\n  \"router_hidden2\": " << h2 << ",\n  \"checksums\": {\n";
    for (size_t i = 0; i < sums.size(); ++i)
      m << "    \"" << sums[i].first << "\": \"" << sums[i].second << "\"" << (i + 1 < sums.size() ? "," : "") << "\n";
    m << "  }\n}\n";
    if (!m) throw IoError{"write failed: meta.json"};
  } catch (const IoError& e) {
    return fail(HNTL_EIO, e.msg);
  } catch (const HipError& e) {
    return fail(e.code == hipErrorOutOfMemory ? HNTL_ENOMEM : HNTL_EDEVICE, e.msg);
  } catch (const std::bad_alloc&) {
    return fail(HNTL_ENOMEM, "host allocation failed");
  }
  return HNTL_OK;
}

extern "C" hntl_status hntl_index_load(const char* dir, hntl_index** out) {
  set_error("");
  if (!dir || !out) return fail(HNTL_EINVAL, "null pointer");
  *out = nullptr;
  hntl_index* h = nullptr;
  try {
    const fs::path p(dir);
    std::ifstream mf(p / "meta.json");
    if (!mf) throw IoError{"cannot read " + (p / "meta.json").string()};
    std::stringstream mss;
    mss << mf.rdbuf();
    const std::string meta = mss.str();
    if (json_str(meta, "format") != "hntl-index") throw IoError{"meta.json is not an hntl index description"};
    if (json_int(meta, "version") != 1) throw IoError{"unknown index file version"};
    const int64_t N = json_int(meta, "N"), d = json_int(meta, "d"), G = json_int(meta, "G"), r = json_int(meta, "r");
    const uint32_t mask = (uint32_t)json_int(meta, "codes_mask");
    if (N <= 0 || d <= 0 || G <= 0 || r <= 0 || G > N || N >= (1ll << 31)) throw IoError{"meta.json sizes out of range"};
    auto cen = read_all<float>(p, "centroids.npy", "<f4", {G, d}, meta);
    auto bas = read_all<float>(p, "basis.npy", "<f4", {G, r, d}, meta);
    auto off = read_all<int64_t>(p, "offsets.npy", "<i8", {G + 1}, meta);
    auto perm = read_all<int32_t>(p, "perm.npy", "<i4", {N}, meta);
    auto codes = read_all<float>(p, "codes.npy", "<f4", {N, r}, meta);
    auto eps = read_all<float>(p, "eps.npy", "<f4", {N}, meta);
    const hntl_status st = hntl_index_create((uint64_t)N, (uint32_t)d, (uint32_t)G, (uint32_t)r, cen.data(),
                                             bas.data(), off.data(), perm.data(), codes.data(), eps.data(), nullptr,
                                             mask, &h);
    if (st != HNTL_OK) return st;
    Index& ix = h->ix;
    HIP_TRY(hipSetDevice(ix.device));
    if (json_int(meta, "raw_vectors")) {  // streamed to the device in pieces
      NpyReader rx(p / "X.npy", "<f4");
      expect_shape(rx, {N, d}, "X.npy");
      ix.X = dev_alloc<float>(&ix, (size_t)N * d);
      const size_t piece = (size_t)256 << 20;
      std::vector<char> buf(std::min(rx.bytes, piece));
      for (size_t o = 0; o < rx.bytes; o += piece) {
        const size_t n = std::min(piece, rx.bytes - o);
        rx.read(buf.data(), n);
        HIP_TRY(hipMemcpy(reinterpret_cast<char*>(ix.X) + o, buf.data(), n, hipMemcpyHostToDevice));
      }
      if (hex64(rx.h) != json_str(meta, "X.npy")) throw IoError{"checksum mismatch: X.npy"};
    }
    if (json_int(meta, "captured")) {
      auto cap = read_all<double>(p, "captured.npy", "<f8", {G}, meta);
      ix.captured.assign(cap.begin(), cap.end());
    }
    const int64_t h1 = json_int(meta, "router_hidden1"), h2 = json_int(meta, "router_hidden2");
    if (h1 > 0) {
      auto W1 = read_all<float>(p, "router_W1.npy", "<f4", {h1, d}, meta);
      auto b1 = read_all<float>(p, "router_b1.npy", "<f4", {h1}, meta);
      auto W2 = read_all<float>(p, "router_W2.npy", "<f4", {h2, h1}, meta);
      auto b2 = read_all<float>(p, "router_b2.npy", "<f4", {h2}, meta);
      auto W3 = read_all<float>(p, "router_W3.npy", "<f4", {G, h2}, meta);
      auto b3 = read_all<float>(p, "router_b3.npy", "<f4", {G}, meta);
      auto mu = read_all<float>(p, "router_mean.npy", "<f4", {d}, meta);
      auto sd = read_all<float>(p, "router_std.npy", "<f4", {d}, meta);
      const hntl_status rs = hntl_router_set(h, (uint32_t)h1, (uint32_t)h2, W1.data(), b1.data(), W2.data(), b2.data(),
                                             W3.data(), b3.data(), mu.data(), sd.data());
      if (rs != HNTL_OK) {
        hntl_index_free(h);
        return rs;
      }
    }
  } catch (const IoError& e) {
    hntl_index_free(h);
    return fail(HNTL_EIO, e.msg);
  } catch (const std::bad_alloc&) {
    hntl_index_free(h);
    return fail(HNTL_ENOMEM, "host allocation failed");
  } catch (const std::exception& e) {  // number parsing in a malformed header
    hntl_index_free(h);
    return fail(HNTL_EIO, std::string("malformed index files: ") + e.what());
  } catch (const HipError& e) {
    hntl_index_free(h);
    return fail(e.code == hipErrorOutOfMemory ? HNTL_ENOMEM : HNTL_EDEVICE, e.msg);
  }
  *out = h;
  return HNTL_OK;
}
