// C ABI of the batched ragged GGDT: plan (validation, workgroup split, device
// tables), run (one persistent launch), destroy.
#include <math.h>
#include <stdlib.h>
#include <string.h>

#include <vector>

#include "ggdt.h"
#include "ggdt_api_internal.h"
#include "ggdt_internal.h"

struct ggdt_plan {
  int n = 0;
  int kclass = 0;
  bool rec = false;
  bool any_classify = false;
  int grid = 0;
  size_t lds = 0;
  size_t ws_bytes = 0;
  ggdt::BatchInst* d_insts = nullptr;
  ggdt::PassDesc* d_passes = nullptr;
  std::vector<ggdt_instance> inst;
  std::vector<ggdt::BatchInst> h_insts;
  std::vector<int> nwg;
  std::vector<long long> npix;
  // backward tables (when every instance has records and gradient buffers)
  bool has_bwd = false;
  int bclass = 0;
  int bgrid = 0;
  size_t blds = 0;
  size_t fwd_ws = 0;
  size_t reset_bytes = 0;  // the header, class words, counters and exchange words: cleared by each run
  ggdt::BatchInst* d_binsts = nullptr;
  ggdt::BwdDesc* d_bpasses = nullptr;
};

namespace ggdt {
namespace {

constexpr size_t kAlign = 256;
size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Cost of an instance with w workgroups, in units of one strided 3D plane
// step of one tile: over the passes, planes times the tiles each workgroup
// walks (ceil(tiles / w)) times the step's weight, plus a per-chunk exchange
// term; layout changes count per round of K tiles a workgroup moves.  Fitted to
// per-pass durations in a 64-instance batch on MI355X (1.26 us per strided 3D
// plane step of a tile and 0.23 us per chunk; 2.45 us per step when the scan
// axis is the contiguous one; 0.53 us per 2D row step and 3.5 us per chunk;
// 3.9 us per round of 4 layout tiles).
double instance_cost(const std::vector<PassDesc>& ps, int w) {
  double c = 0.0;
  for (const PassDesc& d : ps) {
    if (d.op != kOpPass) {
      const double tiles = (double)d.Np * ((d.Nq + 63) / 64) * ((d.Na + 63) / 64);
      c += 3.1 * ceil(tiles / ((double)w * (d.K > 0 ? d.K : 1)));
      continue;
    }
    const int tiles = d.ntp * d.ntq;
    const int per = (tiles + w - 1) / w;
    const bool two_d = d.TP == 1;
    const double step = two_d ? 0.42 : (d.sa == 1 ? 1.9 : 1.0);
    c += step * (double)(d.Na - 1) * per + (two_d ? 2.8 : 0.19) * d.nchunk;
  }
  return c;
}

int max_tiles_of(const std::vector<PassDesc>& ps) {
  int m = 1;
  for (const PassDesc& d : ps) m = d.ntp * d.ntq > m ? d.ntp * d.ntq : m;
  return m;
}

// Exchange words one parity slot of an instance needs: tiles x tile cells, for
// the forward passes' tiles and for the reverse passes' (16 x 16 in 3D, 256
// in 2D), which reuse the instance's exchange area.
size_t max_cells_of(const std::vector<PassDesc>& ps) {
  size_t m = 1;
  for (const PassDesc& d : ps) {
    const size_t fwd = (size_t)d.ntp * d.ntq * d.TP * d.TQ;
    const size_t bwd = d.TP == 1 ? (size_t)((d.Nq + kTQ2 - 1) / kTQ2) * kTQ2
                                 : (size_t)((d.Np + kTP3 - 1) / kTP3) * ((d.Nq + kTQ3 - 1) / kTQ3) * kTP3 * kTQ3;
    m = fwd > m ? fwd : m;
    m = bwd > m ? bwd : m;
  }
  return m;
}

int validate_instance(const ggdt_instance& in, Problem* pr) {
  if (!in.image || !in.softmask || !in.out) return GGDT_ERR_NULL_PTR;
  int rc = make_problem(in.ndim, in.dims, in.C, pr);
  if (rc) return rc;
  rc = check_params(in.ndim, in.spacing, in.v, in.lambda, in.iterations);
  if (rc) return rc;
  const size_t nb = (size_t)pr->N * 4, ni = (size_t)pr->N * pr->C * 4;
  const void* ins[2] = {in.image, in.softmask};
  const size_t nins[2] = {ni, nb};
  rc = check_alias(in.out, nb, ins, nins, 2);
  if (rc) return rc;
  if (in.records) {
    const size_t nrec = (size_t)in.iterations * 2 * in.ndim * pr->N;
    const void* ins2[3] = {in.image, in.softmask, in.out};
    const size_t nins2[3] = {ni, nb, nb};
    rc = check_alias(in.records, nrec, ins2, nins2, 3);
    if (rc) return rc;
  }
  return GGDT_OK;
}

}  // namespace
}  // namespace ggdt

using namespace ggdt;

extern "C" {

int ggdt_batched_plan(const ggdt_instance* instances, int n, const ggdt_tuning* tuning, ggdt_plan** plan_out,
                      size_t* workspace_bytes) {
  if (!instances || !plan_out || !workspace_bytes) return GGDT_ERR_NULL_PTR;
  if (n < 1) return GGDT_ERR_BAD_SHAPE;
  *plan_out = nullptr;
  std::vector<Problem> prs(n);
  int maxC = 1, maxC2 = 0, maxC3 = 0;
  bool has2d = false, has3d = false, rec = false, any_cls = false;
  for (int i = 0; i < n; ++i) {
    const int rc = validate_instance(instances[i], &prs[i]);
    if (rc) return rc;
    maxC = instances[i].C > maxC ? instances[i].C : maxC;
    has2d |= instances[i].ndim == 2;
    has3d |= instances[i].ndim == 3;
    if (instances[i].ndim == 2) maxC2 = instances[i].C > maxC2 ? instances[i].C : maxC2;
    else maxC3 = instances[i].C > maxC3 ? instances[i].C : maxC3;
    rec |= instances[i].records != nullptr;
    any_cls = true;  // the classification decides every instance's edge-cost mode
  }
  int kclass = maxC <= kBatchMaxC[0] ? 0 : 1;
  const bool wide = tuning && (tuning->tile_p == kBatchTile3[2] || tuning->tile_q == kBatchTile3[2]);
  if (tuning && (tuning->tile_p > 0 || tuning->tile_q > 0) && !wide &&
      !(tuning->tile_p == kBatchTile3[0] || tuning->tile_q == kBatchTile3[0]))
    return GGDT_ERR_BAD_PARAM;
  if (wide) {
    // 24 x 24 volume tiles with K = 4: single-channel batches only
    if (tuning->chunk > 0 && tuning->chunk != kBatchK3[2]) return GGDT_ERR_BAD_PARAM;
    kclass = 2;
  } else if (tuning && tuning->chunk > 0) {
    if (tuning->chunk == kBatchK3[1] || tuning->chunk == kBatchK2[1]) kclass = 1;
    else if (tuning->chunk != kBatchK3[0] && tuning->chunk != kBatchK2[0]) return GGDT_ERR_BAD_PARAM;
  }
  if (maxC > kBatchMaxC[kclass]) return kclass == 0 ? GGDT_ERR_BAD_PARAM : GGDT_ERR_UNSUPPORTED;
  int rc = check_device();
  if (rc) return rc;
  const size_t lds = batched_lds_bytes(kclass, maxC, has2d, has3d);
  if (lds == 0 || lds > kMaxLdsBytes) return GGDT_ERR_UNSUPPORTED;
  int cap = batched_capacity(kclass, rec, lds);
  if (cap <= 0) return GGDT_ERR_HIP;
  if (tuning && tuning->wg_per_cu > 0) {
    int dev = 0, cus = 0;
    if (hipGetDevice(&dev) != hipSuccess || hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev))
      return GGDT_ERR_HIP;
    const int c2 = tuning->wg_per_cu * cus;
    cap = c2 < cap ? c2 : cap;
  }
  if (n > cap) return GGDT_ERR_UNSUPPORTED;

  // Pass descriptors (schedule order) per instance, chunk length of the kernel
  // class.  As in the plain forward, the passes along the last axis of a
  // single-channel volume without records run on scan-major copies of D and
  // of the image in the workspace: layout changes (descriptors with op !=
  // kOpPass) move the image there before the first pass and D there and back
  // around each iteration's last two passes.  Workspace offsets not yet known
  // are marked kSlotD / kSlotImage and filled in with the layout below.
  constexpr long long kSlotD = -2, kSlotImage = -3, kSlotRec = -4;
  std::vector<std::vector<PassDesc>> passes(n);
  std::vector<bool> sm(n, false);
  for (int i = 0; i < n; ++i) {
    const ggdt_instance& in = instances[i];
    const int npass = in.iterations * 2 * in.ndim;
    sm[i] = in.ndim == 3 && in.C == 1 && npass > 0 && scan_major_bytes(prs[i]) > 0 &&
            lds >= (size_t)64 * 65 * 4;  // room for one transpose tile
    const int D0 = prs[i].dims[0], D1 = prs[i].dims[1], D2 = prs[i].dims[2];
    auto layout_op = [&](int op, const void* src, long long src_off, void* dst, long long dst_off, int esz = 4) {
      PassDesc L;
      memset(&L, 0, sizeof L);
      L.op = op;
      L.esz = esz;
      L.rec_off = -1;
      L.image = static_cast<const float*>(src);
      L.image_off = src_off;
      L.D = static_cast<float*>(dst);
      L.d_off = dst_off;
      L.Np = D0;
      L.Nq = D1;
      L.Na = D2;
      // tiles per round: 4 when the launch's LDS holds 4 tiles of 64 x 65 elements, else 1
      L.K = lds >= (size_t)4 * 64 * 65 * esz ? 4 : 1;
      passes[i].push_back(L);
    };
    if (sm[i]) layout_op(kOpToScanMajor, in.image, -1, nullptr, kSlotImage);
    unsigned base = 0;
    for (int p = 0; p < npass; ++p) {
      PassDesc d;
      rc = build_pass(prs[i], in.image, in.softmask, in.spacing, in.v, in.lambda, in.out, in.records, p, base, &d);
      if (rc) return rc;
      d.K = in.ndim == 3 ? kBatchK3[kclass] : kBatchK2[kclass];
      if (in.ndim == 3) {
        d.TP = d.TQ = kBatchTile3[kclass];
        d.ntp = (d.Np + d.TP - 1) / d.TP;
        d.ntq = (d.Nq + d.TQ - 1) / d.TQ;
      }
      d.nchunk = (d.Na - 1 + d.K - 1) / d.K;
      base += (unsigned)d.nchunk + 1u;
      const int k = p % 6;
      if (sm[i] && k == 4) layout_op(kOpToScanMajor, in.out, -1, nullptr, kSlotD);
      uint8_t* rec_c = d.rec;  // this pass's records in the array layout
      if (sm[i] && k >= 4) {
        // planes (z, y) of the [W][D][H] copies: same tiles, offsets and constants
        d.sa = D0 * D1;
        d.sp = D1;
        d.sq = 1;
        d.image = nullptr;
        d.image_off = kSlotImage;
        d.D = nullptr;
        d.d_off = kSlotD;
        if (rec_c) {  // staged scan-major, then moved to the array layout
          d.rec = nullptr;
          d.rec_off = kSlotRec;
        }
      }
      passes[i].push_back(d);
      if (sm[i] && k >= 4 && rec_c) layout_op(kOpFromScanMajor, nullptr, kSlotRec, rec_c, -1, 1);
      if (sm[i] && k == 5) layout_op(kOpFromScanMajor, nullptr, kSlotD, in.out, -1);
    }
  }

  // Split the co-resident workgroups: one each, then greedily to the instance
  // with the largest remaining cost while it has tiles left to spread.
  std::vector<int> w(n, 1);
  std::vector<double> cost(n);
  for (int i = 0; i < n; ++i) cost[i] = instance_cost(passes[i], 1);
  int used = n;
  while (used < cap) {
    int best = -1;
    for (int i = 0; i < n; ++i)
      if (w[i] < max_tiles_of(passes[i]) && !passes[i].empty() && (best < 0 || cost[i] > cost[best])) best = i;
    if (best < 0) break;
    ++w[best];
    cost[best] = instance_cost(passes[best], w[best]);
    ++used;
  }

  // Workspace: header, class words, counters, exchange words per instance.
  ggdt_plan* plan = new ggdt_plan();
  plan->n = n;
  plan->kclass = kclass;
  plan->rec = rec;
  plan->any_classify = any_cls;
  plan->lds = lds;
  plan->inst.assign(instances, instances + n);
  size_t off = (size_t)kHeaderWords * 4;
  const size_t cls_off = off;
  off = align_up(off + (size_t)n * 4);
  const size_t ctr_off = off;
  off = align_up(off + (size_t)n * 4);
  // Exchange words of every instance first (the region each run clears),
  // then the instances' scan-major copies (never cleared: written before read).
  std::vector<PassDesc> flat;
  int wg0 = 0;
  for (int i = 0; i < n; ++i) {
    const ggdt_instance& in = instances[i];
    BatchInst bi;
    memset(&bi, 0, sizeof bi);
    bi.ndim = in.ndim;
    bi.mode = requested_mode(in.lambda, in.C);
    bi.npass = (int)passes[i].size();
    bi.wg0 = wg0;
    bi.nwg = w[i];
    bi.xbuf_off = (long long)off;
    bi.ctr_off = (long long)(ctr_off + 4 * (size_t)i);
    bi.cls_off = (long long)(cls_off + 4 * (size_t)i);
    bi.image = in.image;
    bi.nimg = (long long)prs[i].C * prs[i].N;
    off = align_up(off + (size_t)2 * max_cells_of(passes[i]) * 8);
    wg0 += w[i];
    plan->h_insts.push_back(bi);
  }
  plan->reset_bytes = off;
  for (int i = 0; i < n; ++i) {
    long long slot_d = -1, slot_img = -1, slot_rec = -1;
    if (sm[i]) {
      slot_d = (long long)off;
      slot_img = (long long)(off + scan_major_vol_bytes(prs[i]));
      off = align_up(off + 2 * scan_major_vol_bytes(prs[i]));
      if (instances[i].records) {
        slot_rec = (long long)off;
        off = align_up(off + (size_t)prs[i].N);
      }
    }
    auto resolve = [&](long long o) {
      return o == kSlotD ? slot_d : (o == kSlotImage ? slot_img : (o == kSlotRec ? slot_rec : o));
    };
    plan->h_insts[i].pass0 = (int)flat.size();
    for (PassDesc d : passes[i]) {
      d.image_off = resolve(d.image_off);
      d.d_off = resolve(d.d_off);
      d.rec_off = resolve(d.rec_off);
      flat.push_back(d);
    }
  }
  plan->grid = wg0;
  plan->nwg = w;
  plan->fwd_ws = off;
  for (int i = 0; i < n; ++i) plan->npix.push_back(prs[i].N);

  // Backward tables: reversed passes, workgroups split for the backward kernel,
  // one adjoint scratch buffer per instance after the forward's regions.
  bool want_bwd = maxC <= 8;
  for (int i = 0; i < n; ++i)
    want_bwd = want_bwd && instances[i].records && instances[i].grad_out && instances[i].grad_image &&
               instances[i].grad_softmask;
  size_t boff = off;
  if (want_bwd) {
    const int bclass = (maxC <= 1 && !has2d) ? 0 : 1;
    // (single-channel volumes: room for four tiles of the layout changes)
    const size_t blds0 = batched_bwd_lds_bytes(maxC2, maxC3), lds4 = (size_t)4 * 64 * 65 * 4;
    const size_t blds = bclass == 0 && blds0 < lds4 ? lds4 : blds0;
    int bcap = blds <= kMaxLdsBytes ? batched_bwd_capacity(bclass, blds) : 0;
    if (tuning && tuning->wg_per_cu > 0 && bcap > 0) {
      int dev = 0, cus = 0;
      if (hipGetDevice(&dev) == hipSuccess && hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess)
        bcap = tuning->wg_per_cu * cus < bcap ? tuning->wg_per_cu * cus : bcap;
    }
    if (bcap >= n) {
      std::vector<std::vector<PassDesc>> bgeo(n);
      std::vector<BwdDesc> bflat;
      std::vector<BatchInst> bh;
      std::vector<long long> scratch_off(n);
      for (int i = 0; i < n; ++i) {
        scratch_off[i] = (long long)boff;
        boff = align_up(boff + (size_t)prs[i].N * 4);
      }
      // As in the forward, the reverses of the passes along the last axis of a
      // single-channel volume run on scan-major copies: of the image (once),
      // and per iteration of abar, dL/dI and the two passes' records, moved
      // there before the pair of reverse passes and abar and dL/dI back after.
      const size_t per_tile4 = (size_t)64 * 65 * 4, per_tile1 = (size_t)64 * 65;
      for (int i = 0; i < n; ++i) {
        const ggdt_instance& in = instances[i];
        const int P = in.iterations * 2 * in.ndim;
        const int K = in.ndim == 3 ? (bclass == 0 ? kBwdBatchKCell : kBwdBatchK3) : kBwdBatchK2;
        const bool bsm = bclass == 0 && in.ndim == 3 && in.C == 1 && P > 0 && scan_major_bytes(prs[i]) > 0 &&
                         blds >= per_tile4;
        const int D0 = prs[i].dims[0], D1 = prs[i].dims[1], D2 = prs[i].dims[2];
        const size_t vol4 = align_up((size_t)prs[i].N * 4), vol1 = align_up((size_t)prs[i].N);
        long long s_img = -1, s_a = -1, s_b = -1, s_g = -1, s_r[2] = {-1, -1};
        if (bsm) {
          s_img = (long long)boff;
          s_a = s_img + (long long)vol4;
          s_b = s_a + (long long)vol4;
          s_g = s_b + (long long)vol4;
          s_r[0] = s_g + (long long)vol4;
          s_r[1] = s_r[0] + (long long)vol1;
          boff = (size_t)s_r[1] + vol1;
        }
        auto op = [&](int kind, int esz, const void* src, long long src_off, void* dst, long long dst_off) {
          BwdDesc L;
          memset(&L, 0, sizeof L);
          L.op = kind;
          L.esz = esz;
          L.lsrc = src;
          L.lsrc_off = src_off;
          L.ldst = dst;
          L.ldst_off = dst_off;
          L.image_off = L.rec_off = L.gi_off = L.a_in_off = L.a_out_off = -1;
          L.Np = D0;
          L.Nq = D1;
          L.Na = D2;
          L.K = blds >= 4 * (esz == 4 ? per_tile4 : per_tile1) ? 4 : 1;
          PassDesc geo{};
          geo.op = kind;
          geo.Np = D0;
          geo.Nq = D1;
          geo.Na = D2;
          geo.K = L.K;
          bgeo[i].push_back(geo);
          bflat.push_back(L);
        };
        if (bsm) op(kOpToScanMajor, 4, in.image, -1, nullptr, s_img);
        unsigned base = 0;
        for (int q = 0; q < P; ++q) {
          const int p = P - 1 - q;
          BwdDesc d;
          rc = build_bwd_pass(prs[i], in.image, in.records, in.spacing, in.lambda, in.grad_image, p, K, base, &d);
          if (rc) {
            ggdt_plan_destroy(plan);
            return rc;
          }
          base += (unsigned)d.nchunk + 1u;
          // abar_in: grad_out, then the previous reversed pass's output; outputs
          // alternate so that the last one lands in grad_softmask.
          const bool out_to_gm = (P - 1 - q) % 2 == 0;
          d.a_out = out_to_gm ? in.grad_softmask : nullptr;
          d.a_out_off = out_to_gm ? -1 : scratch_off[i];
          if (q == 0) {
            d.a_in = in.grad_out;
          } else {
            const bool prev_gm = (P - q) % 2 == 0;
            d.a_in = prev_gm ? in.grad_softmask : nullptr;
            d.a_in_off = prev_gm ? -1 : scratch_off[i];
          }
          const int k = p % 6;
          if (bsm && k == 5) {  // first of the pair (2, -), (2, +) in reverse order
            op(kOpToScanMajor, 4, d.a_in, d.a_in_off, nullptr, s_a);
            op(kOpToScanMajor, 4, in.grad_image, -1, nullptr, s_g);
            op(kOpToScanMajor, 1, in.records + (size_t)p * prs[i].N, -1, nullptr, s_r[0]);
            op(kOpToScanMajor, 1, in.records + (size_t)(p - 1) * prs[i].N, -1, nullptr, s_r[1]);
          }
          const float* out_ptr = d.a_out;
          const long long out_off = d.a_out_off;
          if (bsm && k >= 4) {
            // planes (z, y) of the [W][D][H] copies: same tiles, offsets and constants
            d.sa = D0 * D1;
            d.sp = D1;
            d.sq = 1;
            d.image = nullptr;
            d.image_off = s_img;
            d.rec = nullptr;
            d.rec_off = s_r[k == 5 ? 0 : 1];
            d.gI = nullptr;
            d.gi_off = s_g;
            d.a_in = nullptr;
            d.a_in_off = k == 5 ? s_a : s_b;
            d.a_out = nullptr;
            d.a_out_off = k == 5 ? s_b : s_a;
          }
          PassDesc geo{};
          geo.TP = d.TP;
          geo.TQ = d.TQ;
          geo.Na = d.Na;
          geo.sa = d.sa;
          geo.ntp = d.ntp;
          geo.ntq = d.ntq;
          geo.nchunk = d.nchunk;
          bgeo[i].push_back(geo);
          bflat.push_back(d);
          if (bsm && k == 4) {  // abar and dL/dI back to the array layout
            op(kOpFromScanMajor, 4, nullptr, s_a, const_cast<float*>(out_ptr), out_off);
            op(kOpFromScanMajor, 4, nullptr, s_g, in.grad_image, -1);
          }
        }
      }
      std::vector<int> bw(n, 1);
      std::vector<double> bc(n);
      for (int i = 0; i < n; ++i) bc[i] = instance_cost(bgeo[i], 1);
      int bused = n;
      while (bused < bcap) {
        int best = -1;
        for (int i = 0; i < n; ++i)
          if (!bgeo[i].empty() && bw[i] < max_tiles_of(bgeo[i]) && (best < 0 || bc[i] > bc[best])) best = i;
        if (best < 0) break;
        ++bw[best];
        bc[best] = instance_cost(bgeo[best], bw[best]);
        ++bused;
      }
      int bwg0 = 0, pass0 = 0;
      for (int i = 0; i < n; ++i) {
        BatchInst bi = plan->h_insts[i];
        bi.npass = (int)bgeo[i].size();
        bi.pass0 = pass0;
        bi.wg0 = bwg0;
        bi.nwg = bw[i];
        pass0 += bi.npass;
        bwg0 += bw[i];
        bh.push_back(bi);
      }
      if (hipMalloc((void**)&plan->d_binsts, sizeof(BatchInst) * n) != hipSuccess ||
          hipMalloc((void**)&plan->d_bpasses, sizeof(BwdDesc) * (bflat.empty() ? 1 : bflat.size())) != hipSuccess ||
          hipMemcpy(plan->d_binsts, bh.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice) != hipSuccess ||
          (!bflat.empty() && hipMemcpy(plan->d_bpasses, bflat.data(), sizeof(BwdDesc) * bflat.size(),
                                       hipMemcpyHostToDevice) != hipSuccess)) {
        ggdt_plan_destroy(plan);
        return GGDT_ERR_HIP;
      }
      plan->has_bwd = true;
      plan->bclass = bclass;
      plan->bgrid = bwg0;
      plan->blds = blds;
    }
  }
  plan->ws_bytes = plan->has_bwd ? boff : off;
  if (hipMalloc((void**)&plan->d_insts, sizeof(BatchInst) * n) != hipSuccess ||
      hipMalloc((void**)&plan->d_passes, sizeof(PassDesc) * (flat.empty() ? 1 : flat.size())) != hipSuccess) {
    ggdt_plan_destroy(plan);
    return GGDT_ERR_HIP;
  }
  if (hipMemcpy(plan->d_insts, plan->h_insts.data(), sizeof(BatchInst) * n, hipMemcpyHostToDevice) != hipSuccess ||
      (!flat.empty() &&
       hipMemcpy(plan->d_passes, flat.data(), sizeof(PassDesc) * flat.size(), hipMemcpyHostToDevice) != hipSuccess)) {
    ggdt_plan_destroy(plan);
    return GGDT_ERR_HIP;
  }
  *plan_out = plan;
  *workspace_bytes = plan->ws_bytes;
  return GGDT_OK;
}

int ggdt_batched_run(const ggdt_plan* plan, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!plan || !workspace) return GGDT_ERR_NULL_PTR;
  if (workspace_bytes < plan->ws_bytes) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  unsigned char* ws = (unsigned char*)workspace;
  if (launch_reset((unsigned*)ws, (long long)(plan->reset_bytes / 4), stream) != hipSuccess) return GGDT_ERR_HIP;
  if (plan->any_classify && launch_batched_classify(plan->d_insts, plan->n, ws, stream) != hipSuccess)
    return GGDT_ERR_HIP;
  // instances with zero iterations: D = v * M
  for (const ggdt_instance& in : plan->inst) {
    if (in.iterations == 0) {
      long long nv = 1;
      for (int b = 0; b < in.ndim; ++b) nv *= in.dims[b];
      if (launch_scale(in.softmask, in.v, in.out, nv, stream) != hipSuccess) return GGDT_ERR_HIP;
    }
  }
  prof_before(stream);
  const hipError_t e = launch_batched(plan->kclass, plan->rec, plan->d_insts, plan->n, plan->d_passes, ws, plan->grid,
                                      plan->lds, g_spin_limit, stream);
  prof_after(stream);
  return e == hipSuccess ? GGDT_OK : GGDT_ERR_HIP;
}

int ggdt_batched_backward(const ggdt_plan* plan, void* workspace, size_t workspace_bytes, hipStream_t stream) {
  if (!plan || !workspace) return GGDT_ERR_NULL_PTR;
  if (!plan->has_bwd) return GGDT_ERR_UNSUPPORTED;
  if (workspace_bytes < plan->ws_bytes) return GGDT_ERR_WORKSPACE_TOO_SMALL;
  unsigned char* ws = (unsigned char*)workspace;
  if (launch_reset((unsigned*)ws, (long long)(plan->reset_bytes / 4), stream) != hipSuccess) return GGDT_ERR_HIP;
  if (plan->any_classify && launch_batched_classify(plan->d_insts, plan->n, ws, stream) != hipSuccess)
    return GGDT_ERR_HIP;
  for (int i = 0; i < plan->n; ++i) {
    const ggdt_instance& in = plan->inst[i];
    if (launch_reset((unsigned*)in.grad_image, plan->npix[i] * in.C, stream) != hipSuccess) return GGDT_ERR_HIP;
    if (in.iterations == 0 && launch_scale(in.grad_out, in.v, in.grad_softmask, plan->npix[i], stream) != hipSuccess)
      return GGDT_ERR_HIP;
  }
  prof_before(stream);
  const hipError_t e = launch_batched_bwd(plan->bclass, plan->d_binsts, plan->n, plan->d_bpasses, ws, plan->bgrid,
                                          plan->blds, g_spin_limit, stream);
  prof_after(stream);
  if (e != hipSuccess) return GGDT_ERR_HIP;
  for (int i = 0; i < plan->n; ++i) {
    const ggdt_instance& in = plan->inst[i];
    if (in.iterations > 0 &&
        launch_scale(in.grad_softmask, in.v, in.grad_softmask, plan->npix[i], stream) != hipSuccess)
      return GGDT_ERR_HIP;
  }
  return GGDT_OK;
}

int ggdt_plan_info(const ggdt_plan* plan, int* n, int* grid, int* bwd_grid, size_t* lds, size_t* bwd_lds) {
  if (!plan) return GGDT_ERR_NULL_PTR;
  if (n) *n = plan->n;
  if (grid) *grid = plan->grid;
  if (bwd_grid) *bwd_grid = plan->has_bwd ? plan->bgrid : 0;
  if (lds) *lds = plan->lds;
  if (bwd_lds) *bwd_lds = plan->has_bwd ? plan->blds : 0;
  return GGDT_OK;
}

void ggdt_plan_destroy(ggdt_plan* plan) {
  if (!plan) return;
  if (plan->d_insts) (void)hipFree(plan->d_insts);
  if (plan->d_passes) (void)hipFree(plan->d_passes);
  if (plan->d_binsts) (void)hipFree(plan->d_binsts);
  if (plan->d_bpasses) (void)hipFree(plan->d_bpasses);
  delete plan;
}

}  // extern "C"
