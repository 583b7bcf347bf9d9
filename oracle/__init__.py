"""CPU oracle for the multi-component sparse kernels.  TEST INFRASTRUCTURE ONLY.

``ref``   -- ctypes front end of the scalar C reference (same operation sequences as
             the method, written independently of the GPU library).
``exact`` -- exact integer/rational arithmetic: exact products, error bounds.

Nothing in the GPU library or its Python binding imports this package.
"""
