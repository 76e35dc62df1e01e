"""Host check of the direct-to-LDS staging layout of the FP64 128 x 128
matrix-core tile (csrc/htlr_core_mfma.hip, core apply of Alg. 4.2).

The kernel's index arithmetic is restated here: 256 threads stage a
128-row x 16-element K slice of each operand with 4 loads each, lane l of
wave w writing 16-byte chunk i*256 + 64*w + l of the unpadded buffer; the
MFMA operand reads address element (row, k) through the XOR swizzle of the
chunk index by (row / 2) mod 8.  Checked: the writes cover the buffer once,
every read returns the element it asks for, and each half-wave of a 64-bit
operand read touches all 64 four-byte LDS banks once (no conflicts).
"""
import numpy as np

NT, E, KBE, BM = 256, 2, 16, 128   # threads, doubles per chunk, K per stage, rows


def staged():
    src = np.arange(BM * KBE).reshape(BM, KBE)
    lds = -np.ones(BM * KBE, dtype=np.int64)
    for i in range(BM // (NT // 8)):
        for tid in range(NT):
            srow, part = tid >> 3, tid & 7
            cpart = part ^ ((srow >> 1) & 7)      # chunk this thread loads
            w, lane = tid >> 6, tid & 63
            q = i * NT + 64 * w + lane             # chunk the load writes
            row = srow + i * (NT // 8)
            for e in range(E):
                assert lds[q * E + e] == -1
                lds[q * E + e] = src[row, cpart * E + e]
    return src, lds


def read_addr(row, lane, kk):
    kc = kk + (lane >> 4)
    sw = (lane >> 1) & 7
    return row * KBE + ((((kc >> 1) ^ sw) << 1) | (kc & 1))


def test_writes_cover_the_buffer_once():
    _, lds = staged()
    assert (lds >= 0).all()


def test_operand_reads_return_their_elements_without_bank_conflicts():
    src, lds = staged()
    for base in (0, 64):                 # rows of the two waves along M (or N)
        for tile in range(4):            # 16-row MFMA tiles of a wave
            for kk in range(0, KBE, 4):
                addrs = []
                for lane in range(64):
                    row = base + tile * 16 + (lane & 15)
                    a = read_addr(row, lane, kk)
                    assert lds[a] == src[row, kk + (lane >> 4)]
                    addrs.append(a)
                for half in range(2):
                    banks = set()
                    for a in addrs[32 * half:32 * (half + 1)]:
                        banks.update({(2 * a) % 64, (2 * a + 1) % 64})
                    assert len(banks) == 64
