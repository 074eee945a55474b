"""CPU FP64 oracle for restarted PDHG on LP.  Test infrastructure only: the
product library never imports, links or runs anything in this package."""
