"""MI355X-native hot path of the conservative cut-cell Navier-Stokes method
(capacities, staggered operators, projection method II with a matrix-free
pressure Poisson solve).  The compute path is libccns.so (HIP, gfx950); this
package only binds it.  Importing the package does not load the library."""

__all__ = ["ccns"]
