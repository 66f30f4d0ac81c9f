"""MI355X-native spatially-varying-kernel image convolution and subtraction.

D = (R (x) K(x,y)) - I with K(x,y) = sum_n sum_m a[n][m] P_m(x,y) B_n,
computed by hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/svconv.h``.  ``svconv`` is the Python binding.
"""
