// Peak candidates of a column range, gathered by one wave while a
// projection kernel produces the spectrum: 64-column windows held across the
// wave's lanes, the peak rule applied to every column whose two neighbours are
// in the range, and a sorted top-k list spread over lanes 0..k-1 with both
// neighbour values of each entry for the refinement (Sec. IV-D.2: the
// candidate of largest cost; the K largest local maxima here).
#pragma once

#include <climits>

#include "peak_rule.h"

namespace ba {

// x of lane l (a wave-uniform lane index), as a scalar
__device__ __forceinline__ float lane_val(float x, int l) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(x), l));
}

// Peak candidates of one column range [g0, gend) (columns at or past the
// candidate rows excluded), kept by one wave; all members are wave-uniform
// except the list entry each lane holds.
struct RangeCands {
  int g0, gend;  // grid sizes stay below 2^30
  int k;
  float lv, ll, lr;  // list entry of this lane: value, left and right neighbour
  int li;            // its grid index (INT_MAX: empty)
  float tv;          // the k-th entry, the bar a new candidate has to pass
  int ti;
  float prev_last;   // value of the column before the current chunk
  float pend_left;   // left neighbour of that column
  bool pend;         // that column waits for its right neighbour
  float e[4];        // P at g0, g0 + 1, gl - 1, gl (gl = gend - 1), clamped to the range

  __device__ void init(int g0_, int gend_, int k_) {
    g0 = g0_;
    gend = gend_;
    k = k_;
    lv = ll = lr = -INFINITY;
    li = INT_MAX;
    tv = -INFINITY;
    ti = INT_MAX;
    prev_last = pend_left = 0.f;
    pend = false;
    e[0] = e[1] = e[2] = e[3] = __int_as_float(0x7fc00000);
  }

  // (v, g) with its neighbours, offered by the whole wave (uniform arguments)
  __device__ void offer(float v, int g, float l, float r, int lane) {
    if (!peak_better(v, g, tv, ti)) return;
    const bool ahead = lane < k && peak_better(lv, li, v, g);
    const int pos = __popcll(__ballot(ahead));  // the list is sorted: the entries ahead are a prefix
    const float sv = __shfl_up(lv, 1, 64), sl = __shfl_up(ll, 1, 64), sr = __shfl_up(lr, 1, 64);
    const int si = __shfl_up(li, 1, 64);
    if (lane == pos) {
      lv = v;
      li = g;
      ll = l;
      lr = r;
    } else if (lane > pos && lane < k) {
      lv = sv;
      li = si;
      ll = sl;
      lr = sr;
    }
    tv = lane_val(lv, k - 1);
    ti = __builtin_amdgcn_readlane(li, k - 1);
  }
};

// Value of lane - 1 (lane + 1) across the whole wave by DPP wave_shr:1
// (wave_shl:1); lane 0 (63) keeps its own value, which callers replace or
// never use.
__device__ __forceinline__ float wave_from_prev_lane(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0x138, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_from_next_lane(float x) {
  return __int_as_float(__builtin_amdgcn_update_dpp(__float_as_int(x), __float_as_int(x), 0x130, 0xf, 0xf, false));
}

// Column t (wave-uniform) of a window whose values lie NPL per lane.
template <int NPL>
__device__ __forceinline__ float window_col(const float (&v)[NPL], int t) {
  if constexpr (NPL == 1) {
    return lane_val(v[0], t);
  } else {
    return (t & 1) ? lane_val(v[1], t >> 1) : lane_val(v[0], t >> 1);
  }
}

// Peak rule over one window of WIN columns starting at wbase, held by the
// wave (column wbase + lane * NPL + i in v[i]; only columns of the range are
// read), then the bookkeeping for the next window.
template <int WIN, int NPL>
__device__ __forceinline__ void window_candidates(RangeCands& rc, const float (&v)[NPL], int wbase, bool first,
                                                  int lane) {
  if (rc.gend <= rc.g0) return;
  // the deferred last column of the previous window meets its right neighbour
  if (rc.pend) {
    const float r0 = lane_val(v[0], 0);
    if (rc.prev_last == rc.prev_last && rc.prev_last > rc.pend_left && rc.prev_last >= r0)
      rc.offer(rc.prev_last, wbase - 1, rc.pend_left, r0, lane);
  }
  float lft[NPL], rgt[NPL];
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    lft[i] = i > 0 ? v[i - 1] : wave_from_prev_lane(v[NPL - 1]);
    rgt[i] = i < NPL - 1 ? v[i + 1] : wave_from_next_lane(v[0]);
  }
  if (lane == 0) lft[0] = rc.prev_last;
#pragma unroll
  for (int i = 0; i < NPL; ++i) {
    const int t = lane * NPL + i;
    const int g = wbase + t;
    // both neighbours inside the range, the right one inside this window
    const bool inner = t < WIN - 1 && g > rc.g0 && g + 1 < rc.gend;
    const bool ok = inner && v[i] == v[i] && v[i] > lft[i] && v[i] >= rgt[i];
    uint64_t m = __ballot(ok);
    while (m) {
      const int src = __builtin_ctzll(m);
      m &= m - 1;
      rc.offer(lane_val(v[i], src), wbase + src * NPL + i, lane_val(lft[i], src), lane_val(rgt[i], src), lane);
    }
  }
  // values at the two ends of the range for the merge
  const int gl = rc.gend - 1;
  if (first) {
    rc.e[0] = window_col<NPL>(v, rc.g0 - wbase);
    rc.e[1] = gl > rc.g0 ? window_col<NPL>(v, rc.g0 + 1 - wbase) : rc.e[0];
  }
  if (gl >= wbase && gl < wbase + WIN) {
    rc.e[3] = window_col<NPL>(v, gl - wbase);
    rc.e[2] = gl == rc.g0 ? rc.e[3] : (gl - 1 >= wbase ? window_col<NPL>(v, gl - 1 - wbase) : rc.prev_last);
  }
  const int gt = wbase + WIN - 1;
  rc.pend = gt > rc.g0 && gt + 1 < rc.gend;
  rc.pend_left = window_col<NPL>(v, WIN - 2);
  rc.prev_last = window_col<NPL>(v, WIN - 1);
}

// The two end columns of a range that is the whole candidate row [0, rows)
// (one wave covers the trial): each is tested against its neighbours with the
// row's wrap, from the end values the window pass kept, and offered to the
// list. After this the list is the trial's top-k.
__device__ __forceinline__ void finish_whole_row(RangeCands& rc, int rows, int wrap0, int lane) {
  if (rc.gend <= rc.g0) return;
  const float pf = rc.e[0], p1 = rc.e[1], pl2 = rc.e[2], pl = rc.e[3];
  // first column: right neighbour p1 (the last column itself when rows == 1)
  {
    bool ok = pf == pf;
    float l = 0.f, r = 0.f;
    if (wrap0) {
      l = pl;
      ok = ok && pf > l;
    }
    if (rows > 1 || wrap0) {
      r = rows > 1 ? p1 : pf;
      ok = ok && pf >= r;
    }
    if (ok) rc.offer(pf, 0, l, r, lane);
  }
  if (rows > 1) {
    bool ok = pl == pl;
    const float l = pl2;
    float r = 0.f;
    ok = ok && pl > l;
    if (wrap0) {
      r = pf;
      ok = ok && pl >= r;
    }
    if (ok) rc.offer(pl, rows - 1, l, r, lane);
  }
}

}  // namespace ba
