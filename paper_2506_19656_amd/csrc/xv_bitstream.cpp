// xv_bitstream.cpp -- host side of the Exp-Golomb bitstream: xv_pack
// (scan of the per-block bit counts, header, payload write) and xv_unpack
// (header checks, parse).
#include <string.h>

#include "xv_host.h"

using namespace xv;
using namespace xv::host;

struct xv_packed {
  void* mem;
  uint64_t bytes;
  uint64_t payload_bits;
  hipStream_t stream;
};

namespace {

constexpr char kPackMagic[8] = {'X', 'V', 'P', 'A', 'C', 'K', '0', '1'};

size_t align256(size_t v) { return (v + 255) & ~(size_t)255; }

BitsArgs bits_args_of(const xv_encoded* e) {
  BitsArgs a{};
  a.N = e->N;
  a.Hb = e->Hb;
  a.Wb = e->Wb;
  a.T = (int32_t)e->T;
  a.gop = e->p.gop;
  a.imodes = (e->p.flags & XV_FLAG_INTRA) != 0;
  a.nunits = (int64_t)e->G * e->T * 4 * e->Hb * e->Wb;
  return a;
}

}  // namespace

extern "C" {

int xv_pack(const xv_encoded* e, void* hip_stream, xv_packed** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  if (!e) return fail(XV_EINVAL, "null encoded cube");
  hipStream_t s = (hipStream_t)hip_stream;
  BitsArgs a = bits_args_of(e);
  a.cbits = e->cbits;
  a.mbits = e->mbits;
  a.levels = e->levels;
  a.mvs = e->mvs;
  a.splits = e->splits;
  const int64_t nb = bits_scan_blocks(a.nunits);
  void* scratch = nullptr;
  XV_HIP(dev_alloc(&scratch, (size_t)(nb + 1) * 8, s), "device allocation of the scan buffer");
  a.block_off = (uint64_t*)scratch;
  a.total = a.block_off + nb;
  uint64_t total = 0;
  hipError_t he = launch_bits_scan(a, s);
  if (he == hipSuccess) he = hipMemcpyAsync(&total, a.total, 8, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  if (he != hipSuccess) {
    dev_free(scratch, s);
    return hip_fail(he, "bitstream scan");
  }
  const uint64_t nseg = (uint64_t)(a.nunits / a.Wb);
  const uint64_t nwords = (total + 31) / 32 + 2;  // two words of padding for readers
  PackHeader h;
  memset(&h, 0, sizeof h);
  memcpy(h.magic, kPackMagic, 8);
  h.version = 1;
  h.header_bytes = sizeof(PackHeader);
  h.T = e->T;
  h.H = e->H;
  h.W = e->W;
  h.bands = e->bands;
  h.src_dtype = e->src_dtype;
  h.G = e->G;
  h.N = e->N;
  h.Hp = e->Hp;
  h.Wp = e->Wp;
  h.Hb = e->Hb;
  h.Wb = e->Wb;
  h.params = e->p;
  h.nseg = nseg;
  h.payload_bits = total;
  h.nwords = nwords;
  h.off_span = align256(sizeof(PackHeader));
  h.span_bytes = e->span_bytes;
  h.off_index = align256(h.off_span + h.span_bytes);
  h.off_payload = align256(h.off_index + nseg * 8);
  h.total_bytes = h.off_payload + nwords * 4;
  xv_packed* pk = new (std::nothrow) xv_packed();
  if (!pk) {
    dev_free(scratch, s);
    return fail(XV_ENOMEM, "host allocation failed");
  }
  pk->bytes = h.total_bytes;
  pk->payload_bits = total;
  pk->stream = s;
  he = dev_alloc(&pk->mem, h.total_bytes, s);
  if (he != hipSuccess) {
    delete pk;
    dev_free(scratch, s);
    return hip_fail(he, "device allocation of the serialised cube");
  }
  char* m = (char*)pk->mem;
  a.index = (uint64_t*)(m + h.off_index);
  a.words = (uint32_t*)(m + h.off_payload);
  he = launch_write_header(h, m, s);
  if (he == hipSuccess)
    he = hipMemcpyAsync(m + h.off_span, e->span, e->span_bytes, hipMemcpyDeviceToDevice, s);
  if (he == hipSuccess) he = launch_fill_u32(a.words, 0u, (int64_t)nwords, s);
  if (he == hipSuccess) {
    ProfScope ps(XV_K_BITS_WRITE, s, (double)total / 8.0);
    he = launch_bits_write(a, s);
  }
  dev_free(scratch, s);
  if (he != hipSuccess) {
    dev_free(pk->mem, s);
    delete pk;
    return hip_fail(he, "bitstream write");
  }
  *out = pk;
  return XV_OK;
}

int xv_packed_view(const xv_packed* p, const void** data, uint64_t* bytes, uint64_t* payload_bits) {
  if (!p) return fail(XV_EINVAL, "null packed cube");
  if (data) *data = p->mem;
  if (bytes) *bytes = p->bytes;
  if (payload_bits) *payload_bits = p->payload_bits;
  return XV_OK;
}

void xv_packed_free(xv_packed* p) {
  if (!p) return;
  if (p->mem) dev_free(p->mem, p->stream);
  delete p;
}

int xv_unpack(const void* data, uint64_t bytes, void* hip_stream, xv_encoded** out) {
  if (!out) return fail(XV_EINVAL, "null output handle");
  *out = nullptr;
  if (!data || bytes < sizeof(PackHeader)) return fail(XV_EINVAL, "buffer too small for a header");
  hipStream_t s = (hipStream_t)hip_stream;
  PackHeader h;
  XV_HIP(hipMemcpyAsync(&h, data, sizeof h, hipMemcpyDeviceToHost, s), "copy header");
  XV_HIP(hipStreamSynchronize(s), "synchronise header copy");
  if (memcmp(h.magic, kPackMagic, 8) != 0 || h.version != 1 || h.header_bytes != sizeof h)
    return fail(XV_EINVAL, "not a serialised cube (bad magic or version)");
  xv_cube cube{(void*)data, h.src_dtype, 0, h.T, h.H, h.W, h.bands};
  int rc = check_cube(&cube, "serialised cube");
  if (rc != XV_OK) return rc;
  if ((rc = check_params(&h.params)) != XV_OK) return rc;
  xv_encoded* e = new (std::nothrow) xv_encoded();
  if (!e) return fail(XV_ENOMEM, "host allocation failed");
  memset(e, 0, sizeof *e);
  dims_of(e, &cube, &h.params);
  e->stream = s;
  BitsArgs a = bits_args_of(e);
  const uint64_t nseg = (uint64_t)(a.nunits / a.Wb);
  const EncLayout lay = enc_layout(e);
  // Every offset is bounded by the buffer before it takes part in a sum or
  // a product, so no check below can wrap around 2^64.
  const bool sizes_ok =
      h.total_bytes <= bytes && h.off_span >= sizeof h && h.off_span <= h.total_bytes &&
      h.span_bytes == lay.span_words * 8 && h.span_bytes <= h.total_bytes - h.off_span &&
      h.off_index >= h.off_span + h.span_bytes && h.off_index <= h.total_bytes &&
      h.nseg == nseg && nseg <= (h.total_bytes - h.off_index) / 8 &&
      h.off_payload >= h.off_index + nseg * 8 && h.off_payload <= h.total_bytes &&
      h.payload_bits <= (uint64_t)1 << 62 && h.nwords == (h.payload_bits + 31) / 32 + 2 &&
      h.nwords <= (h.total_bytes - h.off_payload) / 4 &&
      h.total_bytes == h.off_payload + h.nwords * 4;
  if (e->G != h.G || e->N != h.N || e->Hp != h.Hp || e->Wp != h.Wp || e->Hb != h.Hb ||
      e->Wb != h.Wb || !sizes_ok) {
    delete e;
    return fail(XV_EINVAL, "serialised cube header is inconsistent");
  }
  e->phys_nb = lay.phys_nb;
  hipError_t he = dev_alloc(&e->keep, lay.keep, s);
  if (he != hipSuccess) {
    delete e;
    return hip_fail(he, "device allocation of the encoded cube");
  }
  bind_keep(e, lay);
  void* err = nullptr;
  he = dev_alloc(&err, 256, s);
  if (he != hipSuccess) {
    xv_encoded_free(e);
    return hip_fail(he, "device allocation");
  }
  const char* m = (const char*)data;
  a.index = (uint64_t*)(m + h.off_index);
  a.words = (uint32_t*)(m + h.off_payload);
  a.nwords = (int64_t)h.nwords;
  a.total_bits = h.payload_bits;
  a.levels_out = e->levels;
  a.mvs_out = e->mvs;
  a.cbits_out = e->cbits;
  a.mbits_out = e->mbits;
  a.splits_out = e->splits;
  a.err = (uint32_t*)err;
  const int64_t lev_words = (int64_t)e->G * e->T * 3 * e->Hp * e->Wp / 2;
  uint32_t herr = 0;
  he = hipMemcpyAsync(e->span, m + h.off_span, h.span_bytes, hipMemcpyDeviceToDevice, s);
  if (he == hipSuccess) he = launch_fill_u32((uint32_t*)e->levels, 0u, lev_words, s);
  if (he == hipSuccess) he = launch_fill_u32(a.err, 0u, 1, s);
  if (he == hipSuccess) {
    ProfScope ps(XV_K_BITS_PARSE, s, (double)h.payload_bits / 8.0);
    he = launch_bits_parse(a, s);
  }
  if (he == hipSuccess) he = hipMemcpyAsync(&herr, a.err, 4, hipMemcpyDeviceToHost, s);
  if (he == hipSuccess) he = hipStreamSynchronize(s);
  dev_free(err, s);
  if (he != hipSuccess) {
    xv_encoded_free(e);
    return hip_fail(he, "bitstream parse");
  }
  if (herr) {
    xv_encoded_free(e);
    return fail(XV_EINVAL, "payload does not parse as the stored codes");
  }
  *out = e;
  return XV_OK;
}


}  // extern "C"
