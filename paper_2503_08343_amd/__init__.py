"""MI355X GMRF posterior engine: sparse Cholesky, solves, sampling and Takahashi selected
inversion of Q + A^T Q_eps A behind the C ABI in include/gmrf.h (libgmrf.so)."""
