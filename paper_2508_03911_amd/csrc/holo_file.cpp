// .holo files (Sec. IV, Holofile system): a 64-byte header, the images as one
// binary stream, an optional JSON footer.  Header fields are little endian;
// the endianness byte describes the pixel data, and 16-bit pixels of a
// big-endian file are swapped on read.  Host-side I/O for file-mode replay.
#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstring>
#include <string>
#include <utility>
#include <vector>

#include "hv.h"
#include "hv_internal.h"

using hvi::fail;

namespace {

void put_le(unsigned char* p, uint64_t v, int n) {
  for (int i = 0; i < n; ++i) p[i] = (unsigned char)(v >> (8 * i));
}
uint64_t get_le(const unsigned char* p, int n) {
  uint64_t v = 0;
  for (int i = 0; i < n; ++i) v |= (uint64_t)p[i] << (8 * i);
  return v;
}

struct File {
  FILE* f = nullptr;
  explicit File(const char* path, const char* mode) : f(std::fopen(path, mode)) {}
  ~File() {
    if (f) std::fclose(f);
  }
};

hv_status read_header(FILE* f, hv_holo_header* h) {
  unsigned char b[64];
  if (std::fread(b, 1, 64, f) != 64) return fail(HV_ERR_ARG, "short .holo header");
  if (std::memcmp(b, "HOLO", 4) != 0) return fail(HV_ERR_ARG, "not a .holo file");
  h->version = (uint16_t)get_le(b + 4, 2);
  h->bits_per_pixel = (uint16_t)get_le(b + 6, 2);
  h->width = (uint32_t)get_le(b + 8, 4);
  h->height = (uint32_t)get_le(b + 12, 4);
  h->image_count = (uint32_t)get_le(b + 16, 4);
  h->data_size = get_le(b + 20, 8);
  h->endianness = b[28];
  h->data_type = b[29];
  if (h->bits_per_pixel != 8 && h->bits_per_pixel != 16)
    return fail(HV_ERR_ARG, ".holo with %u bits per pixel is not supported", (unsigned)h->bits_per_pixel);
  if (h->data_size != (uint64_t)h->width * h->height * h->image_count * (h->bits_per_pixel / 8))
    return fail(HV_ERR_ARG, ".holo data size %llu does not match the image count and size",
                (unsigned long long)h->data_size);
  return HV_OK;
}

}  // namespace

extern "C" {

hv_status hv_holo_read_header(const char* path, hv_holo_header* out, uint64_t* footer_bytes) {
  if (!path || !out) return fail(HV_ERR_ARG, "NULL argument");
  File file(path, "rb");
  if (!file.f) return fail(HV_ERR_ARG, "cannot open %s", path);
  hv_status s = read_header(file.f, out);
  if (s) return s;
  if (footer_bytes) {
    if (std::fseek(file.f, 0, SEEK_END) != 0) return fail(HV_ERR_ARG, "cannot seek %s", path);
    const long end = std::ftell(file.f);
    const uint64_t body = 64 + out->data_size;
    *footer_bytes = (uint64_t)end > body ? (uint64_t)end - body : 0;
  }
  return HV_OK;
}

hv_status hv_holo_read_frames(const char* path, int64_t first, int64_t count, void* host_dst) {
  if (!path || !host_dst) return fail(HV_ERR_ARG, "NULL argument");
  File file(path, "rb");
  if (!file.f) return fail(HV_ERR_ARG, "cannot open %s", path);
  hv_holo_header h;
  hv_status s = read_header(file.f, &h);
  if (s) return s;
  if (first < 0 || count < 0 || first + count > (int64_t)h.image_count)
    return fail(HV_ERR_ARG, "images [%lld, %lld) outside the file's %u", (long long)first,
                (long long)(first + count), (unsigned)h.image_count);
  const uint64_t frame = (uint64_t)h.width * h.height * (h.bits_per_pixel / 8);
  if (std::fseek(file.f, (long)(64 + first * frame), SEEK_SET) != 0) return fail(HV_ERR_ARG, "seek failed");
  const uint64_t bytes = (uint64_t)count * frame;
  if (std::fread(host_dst, 1, bytes, file.f) != bytes) return fail(HV_ERR_ARG, "short .holo data");
  if (h.bits_per_pixel == 16 && h.endianness == 1) {
    unsigned char* p = (unsigned char*)host_dst;
    for (uint64_t i = 0; i + 1 < bytes; i += 2) std::swap(p[i], p[i + 1]);
  }
  return HV_OK;
}

hv_status hv_holo_read_footer(const char* path, char* dst, uint64_t cap) {
  if (!path || !dst) return fail(HV_ERR_ARG, "NULL argument");
  File file(path, "rb");
  if (!file.f) return fail(HV_ERR_ARG, "cannot open %s", path);
  hv_holo_header h;
  hv_status s = read_header(file.f, &h);
  if (s) return s;
  if (std::fseek(file.f, (long)(64 + h.data_size), SEEK_SET) != 0) return fail(HV_ERR_ARG, "seek failed");
  const size_t got = std::fread(dst, 1, cap > 0 ? cap - 1 : 0, file.f);
  if (cap > 0) dst[got] = '\0';
  return HV_OK;
}

hv_status hv_holo_write(const char* path, const hv_holo_header* h, const void* host_frames, const char* footer_json) {
  if (!path || !h || (!host_frames && h->image_count > 0)) return fail(HV_ERR_ARG, "NULL argument");
  if (h->bits_per_pixel != 8 && h->bits_per_pixel != 16) return fail(HV_ERR_ARG, "bits per pixel must be 8 or 16");
  if (h->endianness > 1) return fail(HV_ERR_ARG, "endianness must be 0 or 1");
  const uint64_t bytes = (uint64_t)h->width * h->height * h->image_count * (h->bits_per_pixel / 8);
  unsigned char b[64] = {};
  std::memcpy(b, "HOLO", 4);
  put_le(b + 4, h->version ? h->version : 7, 2);
  put_le(b + 6, h->bits_per_pixel, 2);
  put_le(b + 8, h->width, 4);
  put_le(b + 12, h->height, 4);
  put_le(b + 16, h->image_count, 4);
  put_le(b + 20, bytes, 8);
  b[28] = h->endianness;
  b[29] = h->data_type;
  File file(path, "wb");
  if (!file.f) return fail(HV_ERR_ARG, "cannot create %s", path);
  if (std::fwrite(b, 1, 64, file.f) != 64) return fail(HV_ERR_ARG, "write failed");
  if (h->bits_per_pixel == 16 && h->endianness == 1) {
    const unsigned char* p = (const unsigned char*)host_frames;
    std::vector<unsigned char> tmp(1 << 20);
    for (uint64_t off = 0; off < bytes; off += tmp.size()) {
      const size_t n = (size_t)std::min<uint64_t>(tmp.size(), bytes - off);
      for (size_t i = 0; i + 1 < n; i += 2) {
        tmp[i] = p[off + i + 1];
        tmp[i + 1] = p[off + i];
      }
      if (std::fwrite(tmp.data(), 1, n, file.f) != n) return fail(HV_ERR_ARG, "write failed");
    }
  } else if (bytes && std::fwrite(host_frames, 1, bytes, file.f) != bytes) {
    return fail(HV_ERR_ARG, "write failed");
  }
  if (footer_json) {
    const size_t n = std::strlen(footer_json);
    if (std::fwrite(footer_json, 1, n, file.f) != n) return fail(HV_ERR_ARG, "write failed");
  }
  return HV_OK;
}

}  // extern "C"
