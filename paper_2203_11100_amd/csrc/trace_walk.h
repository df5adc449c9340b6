// Host side of the traceback: the walk back through the per-cell codes of
// the int32 intra-task kernel's traceback variant (k_intra.hip).
#pragma once
#include <stdint.h>

#include <vector>

namespace swdb {

// Walks an optimal local alignment back from its end (0-based q_end,
// db_end) through one sequence's codes ([column][row] bytes, ld bytes per
// column: bits 0-1 where H came from - 0 it is 0, 1 the diagonal, 2 E, 3 F;
// bit 2 E of the next column opens a gap; bit 3 F of the next row opens a
// gap) and appends it, first operation first, as runs (length << 2 | op)
// with op 0 = M, 1 = I (query residue against a gap), 2 = D (database
// residue against a gap).  Sets the 0-based first positions.  Returns false
// on codes that do not form a path.
bool walk_alignment(const uint8_t* dir, int64_t ld, int32_t q_end, int32_t db_end,
                    int32_t* q_begin, int32_t* db_begin, std::vector<uint32_t>* runs);

}  // namespace swdb
