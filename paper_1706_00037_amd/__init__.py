"""MI355X-native hot path of the diversified multi-start UBQP method
(Lewis, arXiv:1706.00037): Glover diversification, exact batched objective on
int8 matrix cores, exact T(lambda) screening, steepest 1-flip ascent, and the
device-resident generation loop, behind the C ABI of include/ubqp.h.

`ubqp` is the ctypes binding of libubqp.so; `inputs` draws seeded synthetic
instances; `build` compiles the HIP sources for gfx950.
"""
