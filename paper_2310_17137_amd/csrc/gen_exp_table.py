"""Print the constants of the table-driven FP64 exponential in kmap64.h:
2^(j/256) for j = 0..255 correctly rounded to FP64 (computed with 60-digit
decimal arithmetic), ln(2)/256 split into a head with 21 trailing zero bits
and a tail, and 256/ln(2). Run: python gen_exp_table.py"""
import struct
from decimal import Decimal, getcontext

N = 256
getcontext().prec = 60
ln2 = Decimal(2).ln()
tab = [float((ln2 * Decimal(j) / Decimal(N)).exp()) for j in range(N)]
c = ln2 / Decimal(N)
bits = struct.unpack("<Q", struct.pack("<d", float(c)))[0] & ~((1 << 21) - 1)
c_hi = struct.unpack("<d", struct.pack("<Q", bits))[0]
c_lo = float(c - Decimal(c_hi))
inv = float(Decimal(N) / ln2)
for i in range(0, N, 4):
    print("    " + ", ".join(x.hex() for x in tab[i:i + 4]) + ",")
print(f"ln2/{N} head {c_hi.hex()}  tail {c_lo.hex()}  {N}/ln2 {inv.hex()}")
