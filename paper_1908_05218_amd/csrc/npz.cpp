// h2_save / h2_load_file: the flat interchange layout as a NumPy .npz file
// (a zip archive of stored, uncompressed .npy members named after the
// arrays), the format numpy.savez writes and numpy.load reads, so matrices
// move between the library and NumPy code unchanged.
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "internal.h"

namespace h2 {

h2_status load_impl(h2_ctx ctx, const h2_host_matrix* m, bool device_blocks, h2_mat* out);

namespace {

uint32_t crc32(const unsigned char* p, size_t n, uint32_t crc = 0) {
  static uint32_t table[256];
  static bool init = false;
  if (!init) {
    for (uint32_t i = 0; i < 256; ++i) {
      uint32_t c = i;
      for (int k = 0; k < 8; ++k) c = (c & 1) ? 0xEDB88320u ^ (c >> 1) : c >> 1;
      table[i] = c;
    }
    init = true;
  }
  crc = ~crc;
  for (size_t i = 0; i < n; ++i) crc = table[(crc ^ p[i]) & 0xff] ^ (crc >> 8);
  return ~crc;
}

struct Array {
  std::string descr;  // '<f8', '<i8', '<i4', '<c16'
  int64_t count = 0;  // elements (shape () counts 1)
  bool scalar = false;
  std::vector<unsigned char> data;
};

void put16(std::vector<unsigned char>& b, uint16_t v) {
  b.push_back(v & 0xff);
  b.push_back(v >> 8);
}
void put32(std::vector<unsigned char>& b, uint32_t v) {
  for (int i = 0; i < 4; ++i) b.push_back((v >> (8 * i)) & 0xff);
}
uint16_t get16(const unsigned char* p) { return (uint16_t)(p[0] | (p[1] << 8)); }
uint32_t get32(const unsigned char* p) {
  return (uint32_t)p[0] | ((uint32_t)p[1] << 8) | ((uint32_t)p[2] << 16) | ((uint32_t)p[3] << 24);
}

// .npy version 1.0 member: magic, header dict padded to a multiple of 64, data
std::vector<unsigned char> npy(const Array& a) {
  std::string h = "{'descr': '" + a.descr + "', 'fortran_order': False, 'shape': " +
                  (a.scalar ? std::string("()") : "(" + std::to_string(a.count) + ",)") + ", }";
  const size_t total = 10 + h.size() + 1;
  h.append((64 - total % 64) % 64, ' ');
  h.push_back('\n');
  std::vector<unsigned char> b = {0x93, 'N', 'U', 'M', 'P', 'Y', 1, 0};
  put16(b, (uint16_t)h.size());
  b.insert(b.end(), h.begin(), h.end());
  b.insert(b.end(), a.data.begin(), a.data.end());
  return b;
}

void write_zip(const std::string& path, const std::vector<std::pair<std::string, Array>>& arrays) {
  FILE* f = std::fopen(path.c_str(), "wb");
  if (!f) throw Error(H2_ERR_ARG, "cannot open " + path + " for writing");
  std::vector<unsigned char> central;
  uint64_t offset = 0;
  auto emit = [&](const std::vector<unsigned char>& b) {
    if (b.size() && std::fwrite(b.data(), 1, b.size(), f) != b.size()) {
      std::fclose(f);
      throw Error(H2_ERR_ARG, "write to " + path + " failed");
    }
    offset += b.size();
  };
  for (const auto& kv : arrays) {
    const std::string name = kv.first + ".npy";
    const std::vector<unsigned char> body = npy(kv.second);
    if (body.size() >= 0xffffffffu || offset >= 0xffffffffu)
      throw Error(H2_ERR_UNSUPPORTED, "npz members and archives are limited to 4 GiB");
    const uint32_t crc = crc32(body.data(), body.size());
    std::vector<unsigned char> lh;
    put32(lh, 0x04034b50);
    put16(lh, 20);
    put16(lh, 0);
    put16(lh, 0);  // stored
    put16(lh, 0);
    put16(lh, 0x21);  // 1980-01-01
    put32(lh, crc);
    put32(lh, (uint32_t)body.size());
    put32(lh, (uint32_t)body.size());
    put16(lh, (uint16_t)name.size());
    put16(lh, 0);
    lh.insert(lh.end(), name.begin(), name.end());
    const uint32_t at = (uint32_t)offset;
    emit(lh);
    emit(body);
    put32(central, 0x02014b50);
    put16(central, 20);
    put16(central, 20);
    put16(central, 0);
    put16(central, 0);
    put16(central, 0);
    put16(central, 0x21);
    put32(central, crc);
    put32(central, (uint32_t)body.size());
    put32(central, (uint32_t)body.size());
    put16(central, (uint16_t)name.size());
    put16(central, 0);
    put16(central, 0);
    put16(central, 0);
    put16(central, 0);
    put32(central, 0);
    put32(central, at);
    central.insert(central.end(), name.begin(), name.end());
  }
  if (offset >= 0xffffffffu) throw Error(H2_ERR_UNSUPPORTED, "npz archives are limited to 4 GiB");
  const uint32_t cd_at = (uint32_t)offset;
  emit(central);
  std::vector<unsigned char> end;
  put32(end, 0x06054b50);
  put16(end, 0);
  put16(end, 0);
  put16(end, (uint16_t)arrays.size());
  put16(end, (uint16_t)arrays.size());
  put32(end, (uint32_t)central.size());
  put32(end, cd_at);
  put16(end, 0);
  emit(end);
  std::fclose(f);
}

// parse one .npy member (version 1.x or 2.x header, little-endian, C order)
Array parse_npy(const unsigned char* p, size_t n, const std::string& name) {
  if (n < 10 || std::memcmp(p, "\x93NUMPY", 6) != 0) throw Error(H2_ERR_ARG, name + ": not a .npy member");
  size_t hl, hs;
  if (p[6] == 1) {
    hl = get16(p + 8);
    hs = 10;
  } else {
    if (n < 12) throw Error(H2_ERR_ARG, name + ": truncated header");
    hl = get32(p + 8);
    hs = 12;
  }
  if (hs + hl > n) throw Error(H2_ERR_ARG, name + ": truncated header");
  const std::string h((const char*)p + hs, hl);
  Array a;
  const size_t d = h.find("'descr'");
  const size_t q1 = h.find('\'', h.find(':', d) + 1), q2 = h.find('\'', q1 + 1);
  if (d == std::string::npos || q1 == std::string::npos || q2 == std::string::npos)
    throw Error(H2_ERR_ARG, name + ": no descr");
  a.descr = h.substr(q1 + 1, q2 - q1 - 1);
  if (h.find("'fortran_order': True") != std::string::npos)
    throw Error(H2_ERR_UNSUPPORTED, name + ": Fortran-ordered member");
  const size_t s = h.find("'shape'");
  const size_t o = h.find('(', s), c = h.find(')', o);
  if (s == std::string::npos || o == std::string::npos || c == std::string::npos)
    throw Error(H2_ERR_ARG, name + ": no shape");
  if (c < o) throw Error(H2_ERR_ARG, name + ": bad shape");
  const std::string dims = h.substr(o + 1, c - o - 1);
  size_t elt = 0;
  if (a.descr == "<f8" || a.descr == "<i8") elt = 8;
  else if (a.descr == "<i4") elt = 4;
  else if (a.descr == "<c16") elt = 16;
  else throw Error(H2_ERR_UNSUPPORTED, name + ": element type " + a.descr);
  // dimensions: comma-separated decimal integers; the product may not exceed
  // what the member's data holds
  const int64_t avail = (int64_t)((n - hs - hl) / elt);
  a.count = 1;
  a.scalar = true;
  int64_t dim = -1;
  for (size_t i = 0; i <= dims.size(); ++i) {
    const char ch = i < dims.size() ? dims[i] : ',';
    if (ch >= '0' && ch <= '9') {
      dim = (dim < 0 ? 0 : dim) * 10 + (ch - '0');
      if (dim > avail) throw Error(H2_ERR_ARG, name + ": truncated data");
    } else if (ch == ',') {
      if (dim >= 0) {
        a.scalar = false;
        a.count = dim == 0 ? 0 : a.count * dim;
        if (a.count > avail) throw Error(H2_ERR_ARG, name + ": truncated data");
      }
      dim = -1;
    } else if (ch != ' ') {
      throw Error(H2_ERR_ARG, name + ": bad shape");
    }
  }
  if (a.count > avail) throw Error(H2_ERR_ARG, name + ": truncated data");
  a.data.assign(p + hs + hl, p + hs + hl + (size_t)a.count * elt);
  return a;
}

std::map<std::string, Array> read_zip(const std::string& path) {
  FILE* f = std::fopen(path.c_str(), "rb");
  if (!f) throw Error(H2_ERR_ARG, "cannot open " + path);
  std::fseek(f, 0, SEEK_END);
  const long size = std::ftell(f);
  std::fseek(f, 0, SEEK_SET);
  std::vector<unsigned char> buf(size > 0 ? (size_t)size : 0);
  if (size <= 0 || std::fread(buf.data(), 1, buf.size(), f) != buf.size()) {
    std::fclose(f);
    throw Error(H2_ERR_ARG, "cannot read " + path);
  }
  std::fclose(f);
  // end of central directory: the last signature within the final 64 KiB
  long e = (long)buf.size() - 22;
  for (; e >= 0 && e >= (long)buf.size() - 65557; --e)
    if (get32(&buf[e]) == 0x06054b50) break;
  if (e < 0 || get32(&buf[e]) != 0x06054b50) throw Error(H2_ERR_ARG, path + ": not a zip archive");
  const uint16_t nent = get16(&buf[e + 10]);
  size_t cd = get32(&buf[e + 16]);
  std::map<std::string, Array> out;
  for (int i = 0; i < nent; ++i) {
    if (cd + 46 > (size_t)e || get32(&buf[cd]) != 0x02014b50 ||
        cd + 46 + get16(&buf[cd + 28]) + get16(&buf[cd + 30]) + get16(&buf[cd + 32]) > (size_t)e)
      throw Error(H2_ERR_ARG, path + ": bad central directory");
    const uint16_t method = get16(&buf[cd + 10]);
    const uint32_t crc = get32(&buf[cd + 16]);
    const uint32_t csize = get32(&buf[cd + 20]), usize = get32(&buf[cd + 24]);
    const uint16_t nl = get16(&buf[cd + 28]), xl = get16(&buf[cd + 30]), cl = get16(&buf[cd + 32]);
    const uint32_t lo = get32(&buf[cd + 42]);
    const std::string name((const char*)&buf[cd + 46], nl);
    if (method != 0) throw Error(H2_ERR_UNSUPPORTED, path + ": compressed member " + name);
    if (csize == 0xffffffffu || usize == 0xffffffffu || lo == 0xffffffffu)
      throw Error(H2_ERR_UNSUPPORTED, path + ": zip64 member " + name);
    if ((size_t)lo + 30 > buf.size() || get32(&buf[lo]) != 0x04034b50)
      throw Error(H2_ERR_ARG, path + ": bad local header");
    const size_t data = (size_t)lo + 30 + get16(&buf[lo + 26]) + get16(&buf[lo + 28]);
    if (data + usize > buf.size()) throw Error(H2_ERR_ARG, path + ": truncated member " + name);
    if (crc32(&buf[data], usize) != crc) throw Error(H2_ERR_ARG, path + ": checksum mismatch in " + name);
    std::string key = name;
    if (key.size() > 4 && key.compare(key.size() - 4, 4, ".npy") == 0) key.resize(key.size() - 4);
    out[key] = parse_npy(&buf[data], usize, name);
    cd += 46 + nl + xl + cl;
  }
  return out;
}

template <typename T>
Array make(const std::vector<T>& v, const char* descr, bool scalar = false) {
  Array a;
  a.descr = descr;
  a.count = (int64_t)v.size();
  a.scalar = scalar;
  a.data.resize(v.size() * sizeof(T));
  if (!v.empty()) std::memcpy(a.data.data(), v.data(), a.data.size());
  return a;
}

}  // namespace
}  // namespace h2

extern "C" {

h2_status h2_save(h2_mat M, const char* path) {
  using namespace h2;
  if (!M || !path) return set_error(H2_ERR_ARG, "null argument");
  try {
    h2_export_sizes sz;
    h2_status st = h2_export_size(M, &sz);
    if (st != H2_OK) return st;
    const int64_t nleaf = (int64_t)1 << sz.L, ncl = ((int64_t)2 << sz.L) - 1;
    const int nc = sz.is_complex ? 2 : 1;
    std::vector<int64_t> leaf_off(nleaf + 1), perm(sz.n), node_off(sz.L + 2), krow(ncl), kcol(ncl),
        V_off(nleaf + 1), W_off(nleaf + 1), Er_off(ncl + 1), Ec_off(ncl + 1), S_off(sz.nnodes + 1),
        F_off(sz.nnodes + 1);
    std::vector<int32_t> row(sz.nnodes), col(sz.nnodes), type(sz.nnodes);
    std::vector<double> V(sz.len_V * nc), W(sz.len_W * nc), Er(sz.len_Er * nc), Ec(sz.len_Ec * nc),
        S(sz.len_S * nc), F(sz.len_F * nc);
    h2_export_buffers b{leaf_off.data(), perm.data(), node_off.data(), row.data(), col.data(),
                        type.data(), krow.data(), kcol.data(), V.data(), W.data(), Er.data(),
                        Ec.data(), S.data(), F.data(), V_off.data(), W_off.data(), Er_off.data(),
                        Ec_off.data(), S_off.data(), F_off.data()};
    st = h2_export(M, &b);
    if (st != H2_OK) return st;
    const char* fd = nc == 2 ? "<c16" : "<f8";
    std::vector<std::pair<std::string, Array>> arrays = {
        {"n", make(std::vector<int64_t>{sz.n}, "<i8", true)},
        {"L", make(std::vector<int64_t>{sz.L}, "<i8", true)},
        {"is_complex", make(std::vector<int64_t>{sz.is_complex}, "<i8", true)},
        {"leaf_off", make(leaf_off, "<i8")}, {"perm", make(perm, "<i8")},
        {"node_off", make(node_off, "<i8")}, {"node_row", make(row, "<i4")},
        {"node_col", make(col, "<i4")}, {"node_type", make(type, "<i4")},
        {"krow", make(krow, "<i8")}, {"kcol", make(kcol, "<i8")},
        {"V", make(V, fd)}, {"V_off", make(V_off, "<i8")}, {"W", make(W, fd)},
        {"W_off", make(W_off, "<i8")}, {"Er", make(Er, fd)}, {"Er_off", make(Er_off, "<i8")},
        {"Ec", make(Ec, fd)}, {"Ec_off", make(Ec_off, "<i8")}, {"S", make(S, fd)},
        {"S_off", make(S_off, "<i8")}, {"F", make(F, fd)}, {"F_off", make(F_off, "<i8")}};
    // complex data: the element count is in complex elements
    for (auto& kv : arrays)
      if (kv.second.descr == "<c16") kv.second.count /= 2;
    write_zip(path, arrays);
    return H2_OK;
  } catch (const Error& e) {
    return set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}

h2_status h2_load_file(h2_ctx ctx, const char* path, h2_mat* out) {
  using namespace h2;
  if (!ctx || !path || !out) return set_error(H2_ERR_ARG, "null argument");
  try {
    std::map<std::string, Array> a = read_zip(path);
    auto need = [&](const char* k, const char* descr) -> const Array& {
      auto it = a.find(k);
      if (it == a.end()) throw Error(H2_ERR_ARG, std::string("missing array ") + k);
      if (it->second.descr != descr) throw Error(H2_ERR_ARG, std::string("array ") + k + " is not " + descr);
      return it->second;
    };
    auto scalar = [&](const char* k) {
      auto it = a.find(k);
      if (it == a.end() || it->second.count != 1 || it->second.data.size() != 8)
        throw Error(H2_ERR_ARG, std::string("missing scalar ") + k);
      int64_t v;
      std::memcpy(&v, it->second.data.data(), 8);
      return v;
    };
    h2_host_matrix m{};
    m.n = scalar("n");
    m.L = scalar("L");
    m.is_complex = a.count("is_complex") ? scalar("is_complex") : 0;
    if (m.L < 0 || m.L > 30 || m.n < 1) return set_error(H2_ERR_ARG, "bad n or L");
    const char* fd = m.is_complex ? "<c16" : "<f8";
    auto i64 = [&](const char* k) { return (const int64_t*)need(k, "<i8").data.data(); };
    auto i32 = [&](const char* k) { return (const int32_t*)need(k, "<i4").data.data(); };
    static const double empty[2] = {0.0, 0.0};
    auto f64 = [&](const char* k) -> const double* {
      const Array& x = need(k, fd);
      return x.count ? (const double*)x.data.data() : empty;
    };
    // sizes the layout implies, checked before any array is read
    const int64_t nleaf = (int64_t)1 << m.L, ncl = ((int64_t)2 << m.L) - 1;
    auto len = [&](const char* k) {
      const std::string key(k);
      const bool i4 = key == "node_row" || key == "node_col" || key == "node_type";
      return need(k, i4 ? "<i4" : "<i8").count;
    };
    if (len("leaf_off") != nleaf + 1 || len("perm") != m.n || len("node_off") != m.L + 2 ||
        len("krow") != ncl || len("kcol") != ncl || len("V_off") != nleaf + 1 ||
        len("W_off") != nleaf + 1 || len("Er_off") != ncl + 1 || len("Ec_off") != ncl + 1)
      return set_error(H2_ERR_ARG, "array sizes do not match n and L");
    const int64_t nnodes = i64("node_off")[m.L + 1];
    if (nnodes < 1 || len("node_row") != nnodes || len("node_col") != nnodes ||
        len("node_type") != nnodes || len("S_off") != nnodes + 1 || len("F_off") != nnodes + 1)
      return set_error(H2_ERR_ARG, "node array sizes do not match node_off");
    // offsets: non-decreasing from 0, ending inside their data array
    auto fits = [&](const char* off, int64_t n_off, const char* data) {
      const int64_t* o = i64(off);
      if (o[0] != 0) return false;
      for (int64_t i = 1; i < n_off; ++i)
        if (o[i] < o[i - 1]) return false;
      return o[n_off - 1] <= need(data, fd).count;
    };
    if (!fits("V_off", nleaf + 1, "V") || !fits("W_off", nleaf + 1, "W") ||
        !fits("Er_off", ncl + 1, "Er") || !fits("Ec_off", ncl + 1, "Ec") ||
        !fits("S_off", nnodes + 1, "S") || !fits("F_off", nnodes + 1, "F"))
      return set_error(H2_ERR_ARG, "offsets run past their arrays");
    m.leaf_off = i64("leaf_off");
    m.perm = i64("perm");
    m.node_off = i64("node_off");
    m.node_row = i32("node_row");
    m.node_col = i32("node_col");
    m.node_type = i32("node_type");
    m.krow = i64("krow");
    m.kcol = i64("kcol");
    m.V = f64("V");
    m.W = f64("W");
    m.Er = f64("Er");
    m.Ec = f64("Ec");
    m.S = f64("S");
    m.F = f64("F");
    m.V_off = i64("V_off");
    m.W_off = i64("W_off");
    m.Er_off = i64("Er_off");
    m.Ec_off = i64("Ec_off");
    m.S_off = i64("S_off");
    m.F_off = i64("F_off");
    return load_impl(ctx, &m, false, out);
  } catch (const Error& e) {
    return set_error(e.code, e.msg);
  } catch (const std::exception& e) {
    return set_error(H2_ERR_INTERNAL, e.what());
  }
}

}  // extern "C"
