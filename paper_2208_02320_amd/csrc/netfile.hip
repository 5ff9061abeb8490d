// hh_net_load: a surrogate network from the .npz file the Python training
// pipeline writes (numpy's savez_compressed: a zip archive of .npy arrays,
// stored or deflated, with zip64 size fields).  Host code only: the archive
// is read with zlib, the arrays are checked against the network's layout, and
// the network is built through the same entry points a caller would use.
#include <zlib.h>

#include <cstdint>
#include <cstdio>
#include <cstring>
#include <map>
#include <string>
#include <vector>

#include "../../include/hh.h"
#include "ctx.hpp"

namespace {

uint32_t rd32(const unsigned char* p) { return p[0] | (p[1] << 8) | (p[2] << 16) | (uint32_t(p[3]) << 24); }
uint16_t rd16(const unsigned char* p) { return uint16_t(p[0] | (p[1] << 8)); }
uint64_t rd64(const unsigned char* p) { return uint64_t(rd32(p)) | (uint64_t(rd32(p + 4)) << 32); }

struct Npy {
  std::string descr;            // e.g. "<f4"
  std::vector<long long> shape;
  std::vector<unsigned char> data;
};

// The members of a zip archive held in memory, decompressed.
std::map<std::string, std::vector<unsigned char>> unzip(const std::vector<unsigned char>& f, std::string& err) {
  std::map<std::string, std::vector<unsigned char>> out;
  if (f.size() < 22) {
    err = "not a zip archive";
    return out;
  }
  // end of central directory: the last signature 0x06054b50 within 64 KiB + 22 of the end
  long long eocd = -1;
  for (long long i = (long long)f.size() - 22; i >= 0 && i >= (long long)f.size() - 65557; --i)
    if (rd32(&f[i]) == 0x06054b50u) {
      eocd = i;
      break;
    }
  if (eocd < 0) {
    err = "zip end-of-central-directory record not found";
    return out;
  }
  uint64_t nent = rd16(&f[eocd + 10]), cd_off = rd32(&f[eocd + 16]);
  if (cd_off == 0xffffffffu || nent == 0xffffu) {
    // zip64 locator just before the record
    if (eocd < 20 || rd32(&f[eocd - 20]) != 0x07064b50u) {
      err = "zip64 locator missing";
      return out;
    }
    const uint64_t z64 = rd64(&f[eocd - 20 + 8]);
    if (z64 + 56 > f.size() || rd32(&f[z64]) != 0x06064b50u) {
      err = "zip64 end record missing";
      return out;
    }
    nent = rd64(&f[z64 + 32]);
    cd_off = rd64(&f[z64 + 48]);
  }
  uint64_t p = cd_off;
  for (uint64_t e = 0; e < nent; ++e) {
    if (p + 46 > f.size() || rd32(&f[p]) != 0x02014b50u) {
      err = "bad zip central directory";
      return {};
    }
    const int method = rd16(&f[p + 10]);
    const uint32_t crc = rd32(&f[p + 16]);
    uint64_t csize = rd32(&f[p + 20]), usize = rd32(&f[p + 24]);
    const int nlen = rd16(&f[p + 28]), xlen = rd16(&f[p + 30]), clen = rd16(&f[p + 32]);
    uint64_t loff = rd32(&f[p + 42]);
    if (p + 46 + nlen + xlen + clen > f.size()) {
      err = "truncated zip central directory";
      return {};
    }
    const std::string name(reinterpret_cast<const char*>(&f[p + 46]), nlen);
    // zip64 extra field: the 64-bit values of the 32-bit fields set to all ones, in order
    for (uint64_t x = p + 46 + nlen; x + 4 <= p + 46 + nlen + xlen;) {
      const int id = rd16(&f[x]), sz = rd16(&f[x + 2]);
      if (id == 1) {
        uint64_t q = x + 4;
        if (usize == 0xffffffffu && q + 8 <= x + 4 + sz) usize = rd64(&f[q]), q += 8;
        if (csize == 0xffffffffu && q + 8 <= x + 4 + sz) csize = rd64(&f[q]), q += 8;
        if (loff == 0xffffffffu && q + 8 <= x + 4 + sz) loff = rd64(&f[q]);
      }
      x += 4 + sz;
    }
    p += 46 + nlen + xlen + clen;
    if (loff + 30 > f.size() || rd32(&f[loff]) != 0x04034b50u) {
      err = "bad zip local header of " + name;
      return {};
    }
    const uint64_t d0 = loff + 30 + rd16(&f[loff + 26]) + rd16(&f[loff + 28]);
    if (d0 + csize > f.size()) {
      err = "truncated zip member " + name;
      return {};
    }
    std::vector<unsigned char> u(usize);
    if (method == 0) {
      if (csize != usize) {
        err = "bad stored member " + name;
        return {};
      }
      std::memcpy(u.data(), &f[d0], usize);
    } else if (method == 8) {
      z_stream zs;
      std::memset(&zs, 0, sizeof(zs));
      if (inflateInit2(&zs, -MAX_WBITS) != Z_OK) {
        err = "zlib init failed";
        return {};
      }
      zs.next_in = const_cast<unsigned char*>(&f[d0]);
      zs.avail_in = uInt(csize);
      zs.next_out = u.data();
      zs.avail_out = uInt(usize);
      const int rc = inflate(&zs, Z_FINISH);
      inflateEnd(&zs);
      if (rc != Z_STREAM_END || zs.total_out != usize) {
        err = "cannot inflate " + name;
        return {};
      }
    } else {
      err = "unsupported zip compression method in " + name;
      return {};
    }
    if (crc32(0L, u.data(), uInt(u.size())) != crc) {
      err = "CRC mismatch in " + name;
      return {};
    }
    out[name] = std::move(u);
  }
  return out;
}

// .npy: magic, version, header length, a Python-literal dict with 'descr',
// 'fortran_order' and 'shape', then the raw data.
bool parse_npy(const std::vector<unsigned char>& b, Npy& a, std::string& err) {
  if (b.size() < 10 || std::memcmp(b.data(), "\x93NUMPY", 6) != 0) {
    err = "not an .npy array";
    return false;
  }
  const int major = b[6];
  size_t hl, h0;
  if (major == 1) {
    hl = rd16(&b[8]);
    h0 = 10;
  } else {
    if (b.size() < 12) return false;
    hl = rd32(&b[8]);
    h0 = 12;
  }
  if (h0 + hl > b.size()) {
    err = "truncated .npy header";
    return false;
  }
  const std::string h(reinterpret_cast<const char*>(&b[h0]), hl);
  auto value_of = [&](const std::string& key) -> std::string {
    const size_t k = h.find("'" + key + "'");
    if (k == std::string::npos) return "";
    size_t v = h.find(':', k);
    if (v == std::string::npos) return "";
    ++v;
    while (v < h.size() && h[v] == ' ') ++v;
    if (h[v] == '\'') {
      const size_t e = h.find('\'', v + 1);
      return h.substr(v + 1, e - v - 1);
    }
    if (h[v] == '(') return h.substr(v, h.find(')', v) - v + 1);
    size_t e = v;
    while (e < h.size() && h[e] != ',' && h[e] != '}') ++e;
    return h.substr(v, e - v);
  };
  a.descr = value_of("descr");
  if (value_of("fortran_order").find("False") == std::string::npos) {
    err = "Fortran-ordered arrays are not read";
    return false;
  }
  const std::string shp = value_of("shape");
  a.shape.clear();
  for (size_t i = 1; i < shp.size();) {
    while (i < shp.size() && (shp[i] < '0' || shp[i] > '9') && shp[i] != ')') ++i;
    if (i >= shp.size() || shp[i] == ')') break;
    long long v = 0;
    while (i < shp.size() && shp[i] >= '0' && shp[i] <= '9') v = v * 10 + (shp[i++] - '0');
    a.shape.push_back(v);
  }
  a.data.assign(b.begin() + h0 + hl, b.end());
  return true;
}

long long count(const Npy& a) {
  long long n = 1;
  for (long long s : a.shape) n *= s;
  return n;
}

}  // namespace

extern "C" int hh_net_load(hh_ctx* ctx, const char* path, hh_net** out) {
  if (!ctx) return HH_EINVAL;
  if (!path || !out) {
    ctx->err = "hh_net_load: path and out are required";
    return HH_EINVAL;
  }
  *out = nullptr;
  FILE* fp = std::fopen(path, "rb");
  if (!fp) {
    ctx->err = std::string("hh_net_load: cannot open ") + path;
    return HH_EINVAL;
  }
  std::vector<unsigned char> f;
  unsigned char buf[1 << 16];
  size_t got;
  while ((got = std::fread(buf, 1, sizeof(buf), fp)) > 0) f.insert(f.end(), buf, buf + got);
  std::fclose(fp);
  std::string err;
  auto members = unzip(f, err);
  if (!err.empty()) {
    ctx->err = "hh_net_load: " + err;
    return HH_EINVAL;
  }
  std::map<std::string, Npy> arr;
  for (const char* k : {"params", "mean", "scale", "fmu", "fsc", "n", "nphase"}) {
    auto it = members.find(std::string(k) + ".npy");
    if (it == members.end() || !parse_npy(it->second, arr[k], err)) {
      ctx->err = std::string("hh_net_load: array ") + k + " missing or unreadable " + err;
      return HH_EINVAL;
    }
  }
  auto want = [&](const char* k, const char* descr, long long n) {
    const Npy& a = arr[k];
    if (a.descr != descr || count(a) != n || (long long)a.data.size() != n * (a.descr[2] - '0')) {
      ctx->err = std::string("hh_net_load: array ") + k + " has type " + a.descr + " and " +
                 std::to_string(count(a)) + " values, expected " + descr + " and " + std::to_string(n);
      return false;
    }
    return true;
  };
  if (!want("n", "<i8", 1) || !want("nphase", "<i8", 1)) return HH_EINVAL;
  long long n = 0, nphase = 0;
  std::memcpy(&n, arr["n"].data.data(), 8);
  std::memcpy(&nphase, arr["nphase"].data.data(), 8);
  if (n < 1 || n > 4096 || nphase < 1 || nphase > 8) {
    ctx->err = "hh_net_load: bad input edge or phase count";
    return HH_EINVAL;
  }
  hh_net* net = nullptr;
  int rc = hh_net_create(ctx, int(nphase), int(n), 0ull, &net);
  if (rc != HH_OK) return rc;
  const long long np = hh_net_num_params(net);
  if (!want("params", "<f4", np) || !want("mean", "<f8", 21) || !want("scale", "<f8", 21) ||
      !want("fmu", "<f8", 8) || !want("fsc", "<f8", 8)) {
    hh_net_destroy(net);
    return HH_EINVAL;
  }
  auto f32 = [&](const char* k) { return reinterpret_cast<const float*>(arr[k].data.data()); };
  auto f64 = [&](const char* k) { return reinterpret_cast<const double*>(arr[k].data.data()); };
  if ((rc = hh_net_set_params(ctx, net, f32("params"), np)) != HH_OK ||
      (rc = hh_net_set_scaling(ctx, net, f64("mean"), f64("scale"))) != HH_OK ||
      (rc = hh_net_set_fraction_scaling(ctx, net, f64("fmu"), f64("fsc"))) != HH_OK) {
    hh_net_destroy(net);
    return rc;
  }
  // optional: interface-density statistics of the training windows
  auto im = members.find("imu.npy"), is = members.find("isc.npy");
  if (im != members.end() && is != members.end()) {
    if (!parse_npy(im->second, arr["imu"], err) || !parse_npy(is->second, arr["isc"], err)) {
      ctx->err = "hh_net_load: arrays imu/isc unreadable " + err;
      hh_net_destroy(net);
      return HH_EINVAL;
    }
    if (!want("imu", "<f8", 1) || !want("isc", "<f8", 1)) {
      hh_net_destroy(net);
      return HH_EINVAL;
    }
    if ((rc = hh_net_set_interface_stats(ctx, net, f64("imu")[0], f64("isc")[0])) != HH_OK) {
      hh_net_destroy(net);
      return rc;
    }
  }
  *out = net;
  return HH_OK;
}
