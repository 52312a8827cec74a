"""MI355X-native k-th eigenvalue of symmetric H^2 matrices (generalized H^2-LDL
inertia + bisection).  The compute path is libh2eig.so (HIP, gfx950); the
Python side only marshals arguments."""
