"""MI355X-native WENO5-Roe compressible Navier-Stokes RHS + RK4 (HIP/gfx950)."""
