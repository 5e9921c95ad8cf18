"""CPU oracle (test infrastructure only; the library never imports it).

``oracle.py`` wraps the plain C FP64 implementation of EVS and VTM;
``tiny.py`` holds dense NumPy forms of the paper's worked examples.
"""
