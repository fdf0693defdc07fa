"""Print the constants of the table-driven FP64 exponential in kmap64.h:
2^(j/64) for j = 0..63 correctly rounded to FP64 (computed with 60-digit
decimal arithmetic), ln(2)/64 split into a head with 21 trailing zero bits and
a tail, and 64/ln(2). Run: python gen_exp_table.py"""
import struct
from decimal import Decimal, getcontext

getcontext().prec = 60
ln2 = Decimal(2).ln()
tab = [float((ln2 * Decimal(j) / Decimal(64)).exp()) for j in range(64)]
c = ln2 / Decimal(64)
bits = struct.unpack("<Q", struct.pack("<d", float(c)))[0] & ~((1 << 21) - 1)
c_hi = struct.unpack("<d", struct.pack("<Q", bits))[0]
c_lo = float(c - Decimal(c_hi))
inv = float(Decimal(64) / ln2)
for i in range(0, 64, 4):
    print("    " + ", ".join(x.hex() for x in tab[i:i + 4]) + ",")
print(f"ln2/64 head {c_hi.hex()}  tail {c_lo.hex()}  64/ln2 {inv.hex()}")
