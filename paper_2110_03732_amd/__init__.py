"""MI355X-native (gfx950, HIP, FP64) library for one implicit-explicit
Runge-Kutta step of resistive GRMHD on a fixed Cartesian grid
(Cheong et al., arXiv:2110.03732).  The compute path is libgrmhd.so
(include/grmhd.h); `grmhd` is its ctypes binding."""
