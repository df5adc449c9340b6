// Host side of the traceback (see trace_walk.h): three states, H, F and E,
// stepping from the end toward the alignment's first matched pair.
#include "trace_walk.h"

#include <stddef.h>

namespace swdb {

bool walk_alignment(const uint8_t* dir, int64_t ld, int32_t q_end, int32_t db_end,
                    int32_t* q_begin, int32_t* db_begin, std::vector<uint32_t>* runs) {
  std::vector<uint8_t> rev;
  int64_t i = (int64_t)q_end + 1, j = (int64_t)db_end + 1;   // 1-based cell
  int state = 0;                                              // 0 H, 1 F, 2 E
  const int64_t bound = 2 * (i + j) + 4;
  for (int64_t step = 0; step <= bound; ++step) {
    if (state != 0 && (i < 1 || j < 1)) return false;
    // H is 0 on the borders (row 0, column 0): the alignment starts there too
    const uint8_t c = state == 0 && (i < 1 || j < 1) ? 0 : dir[(j - 1) * ld + (i - 1)];
    if (state == 0) {
      const int src = c & 3;
      if (src == 0) {
        *q_begin = (int32_t)i;
        *db_begin = (int32_t)j;
        for (size_t x = rev.size(); x-- > 0;) {
          const uint32_t op = rev[x];
          if (!runs->empty() && (runs->back() & 3u) == op) runs->back() += 4u;
          else runs->push_back(4u | op);
        }
        return true;
      }
      if (src == 1) { rev.push_back(0); --i; --j; }
      else state = src == 3 ? 1 : 2;
    } else if (state == 1) {
      rev.push_back(1);
      if (i < 2) return false;
      state = (dir[(j - 1) * ld + (i - 2)] >> 3) & 1 ? 0 : 1;
      --i;
    } else {
      rev.push_back(2);
      if (j < 2) return false;
      state = (dir[(j - 2) * ld + (i - 1)] >> 2) & 1 ? 0 : 2;
      --j;
    }
  }
  return false;
}

}  // namespace swdb
